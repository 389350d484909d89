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
// The cost |x - y|^2 / eps = ch |i - j|^2 is separable, so every log-sum-exp
// over the X tile (lx1 x lx2) or the Y box (L1 x L2) is done as two 1-D passes
// over LDS-resident arrays.  Potentials are kept as an FP64 affine base plus a
// residual array of type R (float or double):
//     beta/eps  = B0 + p . j + b~(j)        (j: box-local index)
//     alpha/eps = A0 + g . i + a~(i)        (i: tile-local index)
// The linear part of the base is folded into the Gaussian kernel by completing
// the square, p . j - ch |j - D|^2 = -ch |j - D - delta|^2 + p . D + ch |delta|^2
// with delta = p / (2 ch), so the FP32 passes only see residuals and kernel
// centres of moderate size while the large affine parts stay in FP64.
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
  static __device__ __forceinline__ float ninf() { return -INFINITY; }
};
template <>
struct M<double> {
  static __device__ __forceinline__ double ex(double x) { return exp(x); }
  static __device__ __forceinline__ double lg(double x) { return log(x); }
  static __device__ __forceinline__ double lg1p(double x) { return log1p(x); }
  static __device__ __forceinline__ double ninf() { return -INFINITY; }
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

// log-sum-exp over n terms  base[k*stride] - ch (k0 + k - c)^2,  k in [0, n).
template <typename R>
__device__ __forceinline__ R lse_gauss(const R* base, int stride, int n, int k0, R c, R ch) {
  R m = M<R>::ninf();
  for (int k = 0; k < n; ++k) {
    const R d = R(k0 + k) - c;
    const R t = base[k * stride] - ch * d * d;
    m = t > m ? t : m;
  }
  R s = R(0);
  for (int k = 0; k < n; ++k) {
    const R d = R(k0 + k) - c;
    s += M<R>::ex(base[k * stride] - ch * d * d - m);
  }
  return m + M<R>::lg(s);
}

// Root of F(v) = logaddexp(A, zt + v) + v/K (convex, increasing) by Newton
// from the upper bound min(-K A, -kappa zt); see eq. proxdiv-problem with
// beta/eps = v - kappa z_aff and q = -beta/lam = c0 - v/K.
template <typename R>
__device__ __forceinline__ R newton_v(R zt, R A, R K, R kappa, R tol, int maxit) {
  const R invK = R(1) / K;
  R v = -kappa * zt;
  const R vb = -K * A;
  v = vb < v ? vb : v;
  for (int it = 0; it < maxit; ++it) {
    const R w = zt + v;
    const R mx = A > w ? A : w;
    const R e = M<R>::ex(-fabs(A - w));
    const R la = mx + M<R>::lg1p(e);   // logaddexp(A, w); A = -inf gives w
    const R F = la + v * invK;
    const R sig = M<R>::ex(w - la);
    const R dv = F / (sig + invK);
    v -= dv;
    if (!(fabs(dv) > tol * (R(1) + fabs(v)))) break;
  }
  return v;
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
  const int cmax = P.cap;   // LDS layout of this problem (allocation covers the largest cap)

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
      d.overflow_any[C.prob] = 1;
    }
    return;
  }
  const int m1 = min(P.margin, (cap - U1) / 2), m2 = min(P.margin, (cap - U2) / 2);
  const int o1 = max(lo1 - m1, 0), o2 = max(lo2 - m2, 0);
  const int L1 = min(hi1 + m1, P.n1) - o1, L2 = min(hi2 + m2, P.n2) - o2;
  const int NY = L1 * L2;

  // ---- LDS carve-up --------------------------------------------------------
  R* bl = reinterpret_cast<R*>(smem_raw);        // b~ + log nu      [cmax^2]
  R* lnv = bl + cmax * cmax;                      // log nu           [cmax^2]
  R* lrr = lnv + cmax * cmax;                     // log r            [cmax^2]
  R* T = lrr + cmax * cmax;                       // X pass 1         [cmax*16]
  R* U0 = T + cmax * kMaxTile;                    // Y pass 1         [16*cmax]
  R* U1a = U0 + cmax * kMaxTile;                  // Y pass 1, half 1 [16*cmax]
  R* al = U1a + cmax * kMaxTile;                  // a~ + log mu      [256]
  R* lnm = al + kBlock;                           // log mu           [256]
  const size_t rbytes = ((size_t)(3 * cmax * cmax + 3 * cmax * kMaxTile + 2 * kBlock) * sizeof(R) + 15) & ~size_t(15);
  double* red = reinterpret_cast<double*>(smem_raw + rbytes);  // 4 waves x 24

  const double eps = P.eps, lam = P.lam, kap = P.kappa, K = P.K, ch = P.ch;
  const R chR = R(ch);
  const int D1 = C.x1 - o1, D2 = C.x2 - o2;      // tile origin in box coordinates
  const double* nu = d.nu + P.grid_off;
  const double* mu = d.mu + P.grid_off;
  const double* Pg = d.P + P.grid_off;

  // ---- X tile inputs -------------------------------------------------------
  const int ti1 = t < lx ? t / lx2 : 0, ti2 = t < lx ? t - ti1 * lx2 : 0;
  const long gx = (long)(C.x1 + ti1) * P.n2 + (C.x2 + ti2);
  double mux = 0.0;
  if (t < lx) {
    mux = mu[gx];
    lnm[t] = R(log(mux));
  }

  // ---- Y box inputs: nu_{-J}, r, log nu, warm start (affine fit) ----------
  double fit[4] = {0.0, 0.0, 0.0, mux};
  for (int o = t; o < NY; o += kBlock) {
    const int j1 = o / L2, j2 = o - j1 * L2;
    const int y1 = o1 + j1, y2 = o2 + j2;
    const long g = (long)y1 * P.n2 + y2;
    const double pv = Pg[g], nv = nu[g];
    double nj = 0.0;
    for (int k = 0; k < C.nb; ++k) {
      const Box b = d.box[C.basic[k]];
      const int a1 = y1 - b.o1, a2 = y2 - b.o2;
      if (a1 >= 0 && a1 < b.l1 && a2 >= 0 && a2 < b.l2)
        nj += d.vals[C.basic[k] * cap2 + (long)a1 * b.l2 + a2];
    }
    const double r = fmax(pv - nj, 0.0) / nv;
    lrr[o] = r > 0.0 ? R(log(r)) : M<R>::ninf();
    lnv[o] = R(log(nv));
    const double f = pv > 0.0 ? -K * log(pv / nv) : 0.0;
    fit[0] += f;
    fit[1] += j1 * f;
    fit[2] += j2 * f;
  }
  block_sum<4>(fit, red);
  const double muJ = fit[3];
  double B0, p1 = 0.0, p2 = 0.0;
  {
    const double N = double(NY), jb1 = 0.5 * (L1 - 1), jb2 = 0.5 * (L2 - 1);
    if (ch > 0.0) {
      if (L1 > 1) p1 = (fit[1] - jb1 * fit[0]) / (L2 * (double)L1 * ((double)L1 * L1 - 1.0) / 12.0);
      if (L2 > 1) p2 = (fit[2] - jb2 * fit[0]) / (L1 * (double)L2 * ((double)L2 * L2 - 1.0) / 12.0);
    }
    B0 = fit[0] / N - p1 * jb1 - p2 * jb2;
  }
  for (int o = t; o < NY; o += kBlock) {
    const int j1 = o / L2, j2 = o - j1 * L2;
    const long g = (long)(o1 + j1) * P.n2 + (o2 + j2);
    const double pv = Pg[g], nv = nu[g];
    const double f = pv > 0.0 ? -K * log(pv / nv) : 0.0;
    bl[o] = R(f - B0 - p1 * j1 - p2 * j2) + lnv[o];
  }
  __syncthreads();

  // ---- X-half: S~(i) = LSE_j [b~ + log nu - ch |j - (D + delta + i)|^2] ----
  auto x_half = [&](double b0, double q1, double q2, double& a0n, double& g1n, double& g2n) -> R {
    const double dl1 = ch > 0.0 ? q1 / (2.0 * ch) : 0.0;
    const double dl2 = ch > 0.0 ? q2 / (2.0 * ch) : 0.0;
    const double c1o = D1 + dl1, c2o = D2 + dl2;
    for (int o = t; o < L1 * lx2; o += kBlock) {
      const int j1 = o / lx2, i2 = o - j1 * lx2;
      T[o] = lse_gauss<R>(bl + j1 * L2, 1, L2, 0, R(c2o + i2), chR);
    }
    __syncthreads();
    R st = R(0);
    if (t < lx) st = lse_gauss<R>(T + ti2, lx2, L1, 0, R(c1o + ti1), chR);
    __syncthreads();
    a0n = -kap * (b0 + q1 * D1 + q2 * D2 + ch * (dl1 * dl1 + dl2 * dl2));
    g1n = -kap * q1;
    g2n = -kap * q2;
    return st;
  };

  // Y pass 1 over columns [ib, ie) of the tile for a given alpha base.
  auto y_pass1 = [&](R* Uo, int ib, int ie, double d2o) {
    for (int o = t; o < lx1 * L2; o += kBlock) {
      const int i1 = o / L2, j2 = o - i1 * L2;
      Uo[o] = lse_gauss<R>(al + i1 * lx2 + ib, 1, ie - ib, ib, R(d2o + j2), chR);
    }
  };

  double A0, g1, g2;
  R at = x_half(B0, p1, p2, A0, g1, g2);
  if (t < lx) {
    at = -R(kap) * at;
    al[t] = at + lnm[t];
  }
  __syncthreads();

  const double tol = P.err * muJ;
  const R newton_tol = sizeof(R) == 8 ? R(1e-14) : R(2e-6);
  const int newton_max = sizeof(R) == 8 ? 100 : 60;
  double B0n = 0.0, pn1 = 0.0, pn2 = 0.0;
  double pxv = 0.0, lpv = 0.0;
  int it = 0;
  bool conv = false;
  for (;;) {
    ++it;
    // ---- Y-half: z~(j) by two passes, then Newton per point ---------------
    const double dq1 = ch > 0.0 ? g1 / (2.0 * ch) : 0.0;
    const double dq2 = ch > 0.0 ? g2 / (2.0 * ch) : 0.0;
    const double d1o = -D1 + dq1, d2o = -D2 + dq2;
    y_pass1(U0, 0, lx2, d2o);
    __syncthreads();
    const double Z0 = A0 - g1 * D1 - g2 * D2 + ch * (dq1 * dq1 + dq2 * dq2);
    for (int o = t; o < NY; o += kBlock) {
      const int j1 = o / L2, j2 = o - j1 * L2;
      const R zt = lse_gauss<R>(U0 + j2, L2, lx1, 0, R(d1o + j1), chR);
      const double c0 = (1.0 - kap) * (Z0 + g1 * j1 + g2 * j2);
      const R A = R(double(lrr[o]) - c0);
      const R v = newton_v<R>(zt, A, R(K), R(kap), newton_tol, newton_max);
      bl[o] = v + lnv[o];
    }
    B0n = -kap * Z0;
    pn1 = -kap * g1;
    pn2 = -kap * g2;
    __syncthreads();

    // ---- next X-half (gives P_X of the pair for the stopping rule) --------
    double A0n, g1n, g2n;
    R atn = x_half(B0n, pn1, pn2, A0n, g1n, g2n);
    double term = 0.0;
    if (t < lx) {
      lpv = (A0 - A0n / kap) + (g1 - g1n / kap) * ti1 + (g2 - g2n / kap) * ti2 + double(at) +
            double(atn);
      const double aol = (A0 + g1 * ti1 + g2 * ti2 + double(at)) / K;   // alpha / lam
      pxv = mux * exp(lpv);
      term = pxv * (lpv + aol) - pxv + mux * exp(-aol);
    }
    double pdv[1] = {term};
    block_sum<1>(pdv, red);
    conv = pdv[0] <= tol;
    const bool done = P.fixed_iters > 0 ? (it >= P.fixed_iters) : (conv || it >= P.max_iter);
    if (done) break;
    A0 = A0n;
    g1 = g1n;
    g2 = g2n;
    if (t < lx) {
      at = -R(kap) * atn;
      al[t] = at + lnm[t];
    }
    __syncthreads();
  }

  // ---- re-split into the basic cells of J --------------------------------
  const double dq1 = ch > 0.0 ? g1 / (2.0 * ch) : 0.0;
  const double dq2 = ch > 0.0 ? g2 / (2.0 * ch) : 0.0;
  const double d1o = -D1 + dq1, d2o = -D2 + dq2;
  const double Z0 = A0 - g1 * D1 - g2 * D2 + ch * (dq1 * dq1 + dq2 * dq2);
  const int nc = lx2 / s;
  y_pass1(U0, 0, s, d2o);
  if (nc > 1) y_pass1(U1a, s, 2 * s, d2o);
  __syncthreads();
  int kr[4], kc[4];
  for (int k = 0; k < C.nb; ++k) {
    const int2 bx = d.basic_xy[C.basic[k]];
    kr[k] = (bx.x - C.x1) / s;
    kc[k] = (bx.y - C.x2) / s;
  }
  // sums: [0..3] <beta, nu_k>, [4..7] |nu_k|, [8..11] <alpha, px>, [12..15] KL terms,
  // [16..19] |mu_k|
  double acc[20];
#pragma unroll
  for (int k = 0; k < 20; ++k) acc[k] = 0.0;
  for (int o = t; o < NY; o += kBlock) {
    const int j1 = o / L2, j2 = o - j1 * L2;
    const long g = (long)(o1 + j1) * P.n2 + (o2 + j2);
    const double v = double(bl[o]) - double(lnv[o]);
    const double c0 = (1.0 - kap) * (Z0 + g1 * j1 + g2 * j2);
    const double beta = eps * (B0n + pn1 * j1 + pn2 * j2 + v);
    const double base = log(nu[g]) + v + c0;
    for (int k = 0; k < C.nb; ++k) {
      const R* Ub = (kc[k] == 0 ? U0 : U1a) + (long)(kr[k] * s) * L2 + j2;
      const R zk = lse_gauss<R>(Ub, L2, s, kr[k] * s, R(d1o + j1), chR);
      const double nt = exp(base + double(zk));
      acc[k] += beta * nt;
      acc[4 + k] += nt;
      d.cand[(long)C.basic[k] * cap2 + o] = nt < P.trunc ? 0.0 : nt;
    }
  }
  if (t < lx) {
    const int k = (ti1 / s) * nc + (ti2 / s);
    const double alpha = eps * (A0 + g1 * ti1 + g2 * ti2 + double(at));
    acc[8 + k] = alpha * pxv;
    acc[12 + k] = mux * (exp(lpv) * lpv - exp(lpv) + 1.0);
    acc[16 + k] = mux;
    d.pxc[P.grid_off + gx] = pxv;
    d.abar[P.grid_off + gx] = alpha;
  }
  block_sum<20>(acc, red);
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
    // exps of the log-sum-exp passes: every Y-half and X-half of the loop, the
    // first X-half, and the re-split passes
    const double xh = (double)L1 * lx2 * L2 + (double)lx * L1;
    const double yh = (double)lx1 * L2 * lx2 + (double)NY * lx1;
    const double rs = (double)lx1 * L2 * lx2 + (double)NY * s * C.nb;
    d.cell_iters[ci] = it;
    d.cell_conv[ci] = conv ? 1 : 0;
    d.cell_bytes[ci] = bytes;
    d.cell_terms[ci] = it * (xh + yh) + xh + rs;
  }
}

size_t cell_lds_bytes(int cap, int precision) {
  const size_t rs = precision == 64 ? 8 : 4;
  const size_t n = 3 * (size_t)cap * cap + 3 * (size_t)cap * kMaxTile + 2 * kBlock;
  size_t bytes = rs * n;
  bytes = (bytes + 15) & ~size_t(15);
  return bytes + sizeof(double) * 4 * 24;
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
