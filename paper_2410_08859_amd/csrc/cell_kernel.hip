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
//     out = s + log sum_k exp(R(base_k - s) - ch (k - c)^2)
// with an FP64 shift s equal to the same output's value at the previous
// Sinkhorn iteration (so the sum is O(1)), the subtraction base_k - s in FP64
// and exp / accumulation in the kernel precision R.  Terms provably below
// e^-W of the output are skipped (window from the row maximum).  When the sum
// leaves [e^-60, e^60] (first iteration, large change) the output is
// recomputed exactly by a max pass and a sum pass.
// The Newton solve works in R on the log cell share relative to the FP64
// reference z/(1+K) (the root when nu_{-J} = 0), finished in FP64.
#include "dd_types.h"

#include <float.h>
#include <limits.h>
#include <math.h>

namespace dduot {

template <typename R>
struct M;
template <>
struct M<float> {
  static __device__ __forceinline__ float ex(float x) { return __expf(x); }
  static __device__ __forceinline__ float lg(float x) { return __logf(x); }
  static __device__ __forceinline__ float lg1p(float x) { return log1pf(x); }
};
template <>
struct M<double> {
  static __device__ __forceinline__ double ex(double x) { return exp(x); }
  static __device__ __forceinline__ double lg(double x) { return log(x); }
  static __device__ __forceinline__ double lg1p(double x) { return log1p(x); }
};

// Sum N doubles over the workgroup in a fixed order (deterministic).
template <int N>
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
    for (int ww = 0; ww < kBlock / 64; ++ww) s += red[ww * N + k];
    v[k] = s;
  }
  __syncthreads();
}

// Y-update, eq. proxdiv-problem, at one point.  With q = -beta/lam,
// q_ref = z/(1+K) (the root when nu_{-J} = 0), a = log r - q_ref and the unknown
// v = -K (q - q_ref) (log of the cell's share of P_Y at the point, up to q_ref),
// the equation reads  G(v) = v + K logaddexp(a, v) = 0;  G is increasing and
// convex, so Newton from any start converges (a step from the left lands right
// of the root, from where the iterates decrease monotonically).  v is O(10), so
// its R rounding is harmless: beta/eps = -K q_ref + v.  In FP32 the root is
// finished by one FP64 Newton step (K logaddexp amplifies FP32 rounding).
template <typename R>
__device__ __forceinline__ double newton_v(double a, double v0, double K, R tol, int maxit) {
  if (!(a > -INFINITY)) return 0.0;
  const R aR = R(a), KR = R(K);
  R v = R(v0);
  for (int it = 0; it < maxit; ++it) {
    R la, sig;
    if (v >= aR) {
      const R e = M<R>::ex(aR - v);
      la = v + M<R>::lg1p(e);
      sig = R(1) / (R(1) + e);
    } else {
      const R e = M<R>::ex(v - aR);
      la = aR + M<R>::lg1p(e);
      sig = e / (R(1) + e);
    }
    const R dv = (v + KR * la) / (R(1) + KR * sig);
    v -= dv;
    if (!(fabs(dv) > tol * (R(1) + fabs(v)))) break;
  }
  double vd = (double)v;
  if (sizeof(R) == 4) {
    double la, sig;
    if (vd >= a) {
      const double e = exp(a - vd);
      la = vd + log1p(e);
      sig = 1.0 / (1.0 + e);
    } else {
      const double e = exp(vd - a);
      la = a + log1p(e);
      sig = e / (1.0 + e);
    }
    vd -= (vd + K * la) / (1.0 + K * sig);
  }
  return vd;
}

// One pass output: LSE over k in [k0, k1) of base[k*stride] - ch (k - c)^2.
// `shift` is an FP64 estimate of the result (have_shift false: none); `bmax`
// bounds base over [k0, k1) from above (window).  Counts exact recomputations
// in nfall.
template <typename R>
__device__ __forceinline__ double lse_pass(const double* base, int stride, int k0, int k1, double c,
                                           double ch, bool have_shift, double shift, double bmax,
                                           double& nfall) {
  constexpr double W = sizeof(R) == 8 ? 745.0 : 104.0;   // e^-W below the R range
  if (have_shift) {
    int a = k0, b = k1;
    if (ch > 0.0) {
      const double r2 = (bmax - shift + W) / ch;
      if (r2 < 0.0) {
        a = b = k0;   // every term is below e^-W of the shift: recompute
      } else {
        const double rr = sqrt(r2);
        a = max(k0, (int)ceil(c - rr));
        b = min(k1, (int)floor(c + rr) + 1);
      }
    }
    R acc = R(0);
    const R cR = R(c), chR = R(ch);
    for (int k = a; k < b; ++k) {
      const R d = R(k) - cR;
      acc += M<R>::ex(R(base[k * stride] - shift) - chR * d * d);
    }
    if (acc > R(8.7e-27) && acc < R(1.1e26)) return shift + (double)M<R>::lg(acc);
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
    const double rr = sqrt((bmax - m + W) / ch);
    a = max(k0, (int)ceil(c - rr));
    b = min(k1, (int)floor(c + rr) + 1);
  }
  R acc = R(0);
  for (int k = a; k < b; ++k) {
    const double d = k - c;
    acc += M<R>::ex(R(base[k * stride] - ch * d * d - m));
  }
  return m + (double)M<R>::lg(acc);
}

template <typename R>
struct CellLds {
  double* bd;    // b(y) = beta/eps + log nu                      [cmax^2]
  double* zp;    // z(y) of the last Y-half                       [cmax^2]
  double* Tt;    // X pass 1 output / re-split half 1             [16*cmax]
  double* Ud;    // Y pass 1 output                               [16*cmax]
  double* Mr;    // row maxima of b                               [cmax]
  double* MU;    // column maxima of Ud                           [cmax]
  double* Mc;    // column maxima of Tt                           [16]
  double* adr;   // a(x) = alpha/eps + log mu                     [256]
  double* Ma;    // row maxima of adr                             [16]
  double* red;   // reductions                                    [4*24]
};

template <typename R>
__host__ __device__ inline size_t cell_lds_layout(int cmax, CellLds<R>* L, unsigned char* base) {
  size_t off = 0;
  auto take = [&](size_t bytes) {
    size_t o = off;
    off = (off + bytes + 15) & ~size_t(15);
    return o;
  };
  const size_t n2 = (size_t)cmax * cmax, nt = (size_t)cmax * kMaxTile;
  size_t o_bd = take(8 * n2), o_zp = take(8 * n2), o_Tt = take(8 * nt), o_Ud = take(8 * nt);
  size_t o_Mr = take(8 * cmax), o_MU = take(8 * cmax), o_Mc = take(8 * kMaxTile);
  size_t o_adr = take(8 * kBlock), o_Ma = take(8 * kMaxTile), o_red = take(8 * 4 * 24);
  if (L) {
    L->bd = (double*)(base + o_bd);
    L->zp = (double*)(base + o_zp);
    L->Tt = (double*)(base + o_Tt);
    L->Ud = (double*)(base + o_Ud);
    L->Mr = (double*)(base + o_Mr);
    L->MU = (double*)(base + o_MU);
    L->Mc = (double*)(base + o_Mc);
    L->adr = (double*)(base + o_adr);
    L->Ma = (double*)(base + o_Ma);
    L->red = (double*)(base + o_red);
  }
  return off;
}

template <typename R>
__global__ __launch_bounds__(kBlock) void k_cell_solve(Dev d, int cell_base) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const int t = threadIdx.x;
  const int ci = cell_base + blockIdx.x;
  const Cell C = d.cells[ci];
  const Prob P = d.probs[C.prob];
  const int cap = P.cap;
  const long cap2 = d.cap2;

  // ---- Y-box of the cell: bbox of the basic boxes, dilated, clipped -------
  int lo1 = INT_MAX, lo2 = INT_MAX, hi1 = INT_MIN, hi2 = INT_MIN;
  for (int k = 0; k < C.nb; ++k) {
    const Box b = d.box[C.basic[k]];
    if (b.l1 > 0 && b.l2 > 0) {
      lo1 = min(lo1, b.o1);
      lo2 = min(lo2, b.o2);
      hi1 = max(hi1, b.o1 + b.l1);
      hi2 = max(hi2, b.o2 + b.l2);
    }
  }
  if (lo1 == INT_MAX) {
    lo1 = C.x1; lo2 = C.x2; hi1 = C.x1 + C.lx1; hi2 = C.x2 + C.lx2;
  }
  const int U1 = hi1 - lo1, U2 = hi2 - lo2;
  const int lx1 = C.lx1, lx2 = C.lx2, lx = lx1 * lx2;
  const int s = P.s;
  if (U1 > cap || U2 > cap) {
    // overflow: keep the old state of every basic cell of J
    for (int k = 0; k < C.nb; ++k) {
      const int b = C.basic[k];
      const Box bx = d.box[b];
      const long n = (long)bx.l1 * bx.l2;
      for (long o = t; o < n; o += kBlock) d.cand[b * cap2 + o] = d.vals[b * cap2 + o];
      if (t == 0) {
        d.cbox[b] = bx;
        d.htil[b] = d.hbar[b];
      }
    }
    if (t < lx) {
      const int i1 = t / lx2, i2 = t - i1 * lx2;
      const long g = P.grid_off + (long)(C.x1 + i1) * P.n2 + (C.x2 + i2);
      d.pxc[g] = d.px[g];
    }
    if (t == 0) {
      d.cell_iters[ci] = -1;
      d.cell_conv[ci] = 0;
      d.cell_bytes[ci] = 0.0;
      d.cell_terms[ci] = 0.0;
      d.cell_fall[ci] = 0.0;
      d.overflow_any[C.prob] = 1;
    }
    return;
  }
  const int m1 = min(P.margin, (cap - U1) / 2), m2 = min(P.margin, (cap - U2) / 2);
  const int o1 = max(lo1 - m1, 0), o2 = max(lo2 - m2, 0);
  const int L1 = min(hi1 + m1, P.n1) - o1, L2 = min(hi2 + m2, P.n2) - o2;
  const int NY = L1 * L2;

  CellLds<R> S;
  cell_lds_layout<R>(cap, &S, smem_raw);
  double* red = S.red;

  const double eps = P.eps, lam = P.lam, kap = P.kappa, K = P.K, ch = P.ch;
  const int D1 = C.x1 - o1, D2 = C.x2 - o2;      // tile origin in box coordinates
  const double* nu = d.nu + P.grid_off;
  const double* mu = d.mu + P.grid_off;
  const double* Pst = d.P + P.grid_off;
  double* wlnv = d.ws_lnv + (long)ci * cap2;
  double* wlrr = d.ws_lrr + (long)ci * cap2;

  // ---- X tile inputs (thread t owns tile point t) --------------------------
  const int ti1 = t < lx ? t / lx2 : 0, ti2 = t < lx ? t - ti1 * lx2 : 0;
  const long gx = (long)(C.x1 + ti1) * P.n2 + (C.x2 + ti2);
  double mux = 0.0, lmux = 0.0;
  if (t < lx) {
    mux = mu[gx];
    lmux = log(mux);
  }

  // ---- Y box inputs: nu_{-J}, r, log nu, warm start -------------------------
  double acc0[2] = {mux, 0.0};
  for (int o = t; o < NY; o += kBlock) {
    const int j1 = o / L2, j2 = o - j1 * L2;
    const int y1 = o1 + j1, y2 = o2 + j2;
    const long g = (long)y1 * P.n2 + y2;
    const double pv = Pst[g], nv = nu[g];
    double nj = 0.0;
    for (int k = 0; k < C.nb; ++k) {
      const Box b = d.box[C.basic[k]];
      const int a1 = y1 - b.o1, a2 = y2 - b.o2;
      if (a1 >= 0 && a1 < b.l1 && a2 >= 0 && a2 < b.l2)
        nj += d.vals[C.basic[k] * cap2 + (long)a1 * b.l2 + a2];
    }
    const double r = fmax(pv - nj, 0.0) / nv;
    acc0[1] += r * nv;
    const double lnv = log(nv);
    wlrr[o] = r > 0.0 ? log(r) : -INFINITY;
    wlnv[o] = lnv;
    // beta^0/eps = -K log(P/nu); b = beta/eps + log nu
    S.bd[o] = (pv > 0.0 ? -K * log(pv / nv) : 0.0) + lnv;
  }
  block_sum<2>(acc0, red);
  const double muJ = acc0[0];
  const double Rmass = acc0[1];   // |nu_{-J}| on the box
  double nfall = 0.0;             // pass outputs recomputed exactly

  // ---- X-half: S(i) = LSE_j [b(j) - ch |j - (D + i)|^2], in place over Tt ----
  // Returns S for the thread's point; sprev is that point's previous S.
  bool have_x = false;
  auto x_half = [&](double sprev) -> double {
    for (int j1 = t; j1 < L1; j1 += kBlock) {
      double m = -INFINITY;
      for (int j2 = 0; j2 < L2; ++j2) m = fmax(m, S.bd[j1 * L2 + j2]);
      S.Mr[j1] = m;
    }
    __syncthreads();
    for (int o = t; o < L1 * lx2; o += kBlock) {
      const int j1 = o / lx2, i2 = o - j1 * lx2;
      S.Tt[o] = lse_pass<R>(S.bd + j1 * L2, 1, 0, L2, (double)(D2 + i2), ch, have_x, S.Tt[o],
                            S.Mr[j1], nfall);
    }
    __syncthreads();
    for (int i2 = t; i2 < lx2; i2 += kBlock) {
      double m = -INFINITY;
      for (int j1 = 0; j1 < L1; ++j1) m = fmax(m, S.Tt[j1 * lx2 + i2]);
      S.Mc[i2] = m;
    }
    __syncthreads();
    double sv = 0.0;
    if (t < lx)
      sv = lse_pass<R>(S.Tt + ti2, lx2, 0, L1, (double)(D1 + ti1), ch, have_x, sprev, S.Mc[ti2],
                       nfall);
    have_x = true;
    __syncthreads();
    return sv;
  };

  double Sx = x_half(0.0);
  double aeps = -kap * Sx;   // alpha/eps of the thread's point

  const double tol = P.err * muJ;
  const R newton_tol = sizeof(R) == 8 ? R(1e-14) : R(1e-6);
  const int newton_max = sizeof(R) == 8 ? 100 : 60;
  double pxv = 0.0, lpv = 0.0;
  int it = 0;
  bool conv = false;
  bool have_y = false;
  double ushift = 0.0;   // shift applied to alpha since the last Y-half (eps units)

  // ---- Y-half pieces -------------------------------------------------------
  auto y_prepare = [&]() {
    if (t < lx) S.adr[t] = aeps + lmux;
    __syncthreads();
    for (int i1 = t; i1 < lx1; i1 += kBlock) {
      double m = -INFINITY;
      for (int i2 = 0; i2 < lx2; ++i2) m = fmax(m, S.adr[i1 * lx2 + i2]);
      S.Ma[i1] = m;
    }
    __syncthreads();
  };
  // Y pass 1 over tile columns [ib, ie): Uo(i1, j2) = LSE_i2 [a - ch (i2 - (j2 - D2))^2]
  auto y_pass1 = [&](double* Uo, int ib, int ie, bool have, double extra) {
    for (int o = t; o < lx1 * L2; o += kBlock) {
      const int i1 = o / L2, j2 = o - i1 * L2;
      Uo[o] = lse_pass<R>(S.adr + i1 * lx2, 1, ib, ie, (double)(j2 - D2), ch, have, Uo[o] + extra,
                          S.Ma[i1], nfall);
    }
    __syncthreads();
    for (int j2 = t; j2 < L2; j2 += kBlock) {
      double m = -INFINITY;
      for (int i1 = 0; i1 < lx1; ++i1) m = fmax(m, Uo[i1 * L2 + j2]);
      S.MU[j2] = m;
    }
    __syncthreads();
  };

  for (;;) {
    ++it;
    if (P.translate) {
      // exact maximisation of the cell dual along (alpha + s, beta - s):
      // e^{s/lam} = (R + sqrt(R^2 + 4AB)) / (2B); FP64 sums (the shift in
      // eps units is K log w, so w must be exact to ~1/K)
      double ab[2] = {0.0, 0.0};
      if (t < lx) ab[0] = mux * exp(-aeps / K);
      for (int o = t; o < NY; o += kBlock) {
        const double lnv = wlnv[o];
        ab[1] += exp(lnv - (S.bd[o] - lnv) / K);
      }
      block_sum<2>(ab, red);
      const double w = (Rmass + sqrt(Rmass * Rmass + 4.0 * ab[0] * ab[1])) / (2.0 * ab[1]);
      const double sh = K * log(w);   // s/eps
      aeps += sh;
      ushift += sh;
      for (int o = t; o < NY; o += kBlock) S.bd[o] -= sh;
      __syncthreads();
    }
    // ---- Y-half: z by two passes, Newton per point --------------------------
    y_prepare();
    y_pass1(S.Ud, 0, lx2, have_y, ushift);
    for (int o = t; o < NY; o += kBlock) {
      const int j1 = o / L2, j2 = o - j1 * L2;
      const double z = lse_pass<R>(S.Ud + j2, L2, 0, lx1, (double)(j1 - D1), ch, have_y,
                                   S.zp[o] + ushift, S.MU[j2], nfall);
      S.zp[o] = z;
      const double lnv = wlnv[o];
      const double qref = z / (K + 1.0);
      // warm start: the previous beta/eps = bd - log nu, i.e. v0 = bd - lnv + K qref
      const double v0 = S.bd[o] - lnv + K * qref;
      const double v = newton_v<R>(wlrr[o] - qref, v0, K, newton_tol, newton_max);
      S.bd[o] = -K * qref + v + lnv;
    }
    have_y = true;
    ushift = 0.0;
    __syncthreads();

    // ---- next X-half (gives P_X of the pair for the stopping rule) ----------
    const double Sn = x_half(Sx);
    double term = 0.0;
    if (t < lx) {
      lpv = aeps + Sn;               // log(P_X / mu)
      const double aol = aeps / K;   // alpha/lam
      pxv = mux * exp(lpv);
      term = pxv * (lpv + aol) - pxv + mux * exp(-aol);
    }
    double pdv[1] = {term};
    block_sum<1>(pdv, red);
    conv = pdv[0] <= tol;
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
  // sums: [0..3] <beta, nu_k>, [4..7] |nu_k|, [8..11] <alpha, px>, [12..15] KL terms,
  // [16..19] |mu_k|, [20] exact recomputations
  double acc[21];
#pragma unroll
  for (int k = 0; k < 21; ++k) acc[k] = 0.0;
  for (int c = 0; c < nc; ++c) {
    double* Uo = c == 0 ? S.Ud : S.Tt;
    y_pass1(Uo, c * s, (c + 1) * s, false, 0.0);
    for (int o = t; o < NY; o += kBlock) {
      const int j1 = o / L2, j2 = o - j1 * L2;
      const double beta = eps * (S.bd[o] - wlnv[o]);
      for (int k = 0; k < C.nb; ++k) {
        if (kc[k] != c) continue;
        const double zk = lse_pass<R>(Uo + j2, L2, kr[k] * s, (kr[k] + 1) * s, (double)(j1 - D1), ch,
                                      true, S.zp[o], S.MU[j2], nfall);
        const double nt = exp(S.bd[o] + zk);   // nu e^{beta/eps} e^{z_k}
        acc[k] += beta * nt;
        acc[4 + k] += nt;
        d.cand[(long)C.basic[k] * cap2 + o] = nt < P.trunc ? 0.0 : nt;
      }
    }
    __syncthreads();
  }
  if (t < lx) {
    const int k = (ti1 / s) * nc + (ti2 / s);
    const double alpha = eps * aeps;
    acc[8 + k] = alpha * pxv;
    acc[12 + k] = mux * (exp(lpv) * lpv - exp(lpv) + 1.0);
    acc[16 + k] = mux;
    d.pxc[P.grid_off + gx] = pxv;
    d.abar[P.grid_off + gx] = alpha;
  }
  acc[20] = nfall;
  block_sum<21>(acc, red);
  if (t == 0) {
    double bytes = 8.0 * (2.0 * NY + 3.0 * lx + (double)C.nb * NY);
    for (int k = 0; k < C.nb; ++k) {
      const int b = C.basic[k];
      const Box ob = d.box[b];
      bytes += 8.0 * ob.l1 * ob.l2;
      d.htil[b] = acc[8 + k] + acc[k] - eps * acc[4 + k] + eps * acc[16 + k] * P.mass_nu +
                  lam * acc[12 + k];
      Box nb;
      nb.o1 = o1; nb.o2 = o2; nb.l1 = L1; nb.l2 = L2;
      d.cbox[b] = nb;
    }
    // log-sum-exp terms of the separable passes: every Y-half and X-half of
    // the loop, the first X-half, and the re-split passes
    const double xh = (double)L1 * lx2 * L2 + (double)lx * L1;
    const double yh = (double)lx1 * L2 * lx2 + (double)NY * lx1;
    const double rs = (double)lx1 * L2 * lx2 + (double)NY * s * C.nb;
    d.cell_iters[ci] = it;
    d.cell_conv[ci] = conv ? 1 : 0;
    d.cell_bytes[ci] = bytes;
    d.cell_terms[ci] = it * (xh + yh) + xh + rs;
    d.cell_fall[ci] = acc[20];
  }
}

size_t cell_lds_bytes(int cap, int precision) {
  if (precision == 64) return cell_lds_layout<double>(cap, nullptr, nullptr);
  return cell_lds_layout<float>(cap, nullptr, nullptr);
}

hipError_t launch_cell_solve(const Dev& d, int cell_base, int ncells, int cap, int precision,
                             hipStream_t st) {
  if (ncells <= 0) return hipSuccess;
  const size_t lds = cell_lds_bytes(cap, precision);
  if (precision == 64) {
    hipLaunchKernelGGL(k_cell_solve<double>, dim3(ncells), dim3(kBlock), lds, st, d, cell_base);
  } else {
    hipLaunchKernelGGL(k_cell_solve<float>, dim3(ncells), dim3(kBlock), lds, st, d, cell_base);
  }
  return hipGetLastError();
}

hipError_t set_cell_lds_limit(size_t bytes) {
  hipError_t e = hipFuncSetAttribute((const void*)k_cell_solve<double>,
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
  if (e != hipSuccess) return e;
  return hipFuncSetAttribute((const void*)k_cell_solve<float>,
                             hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
}

}  // namespace dduot
