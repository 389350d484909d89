// Warm start of a domain-decomposition layer from global dual potentials
// (Sec. 4.4 "Sinkhorn warm start" with the multiscale layers of Sec. 4.4).
//
// The coarse layers are solved by the global Sinkhorn iteration; their
// potentials (alpha, beta), in cost units, are carried to the next layer by
// linear interpolation between the block centres, and the first DD layer
// starts from the plan they define,
//     pi(x, y) = exp((alpha(x) + beta(y) - c(x, y)) / eps) mu(x) nu(y),
// split by basic cells: nu_i(y) = sum_{x in X_i} pi(x, y), scanned over a
// window of Y points per basic cell, entries below the truncation threshold
// dropped, box = bbox of the rest.  Two launches: the boxes (phase 0), then,
// once the host has placed them in the state pool, the values, P_X and the
// tracked pieces (phase 1).  The cell plan is pi on X_i x (kept points of the box);
// P_X pi and the tracked piece
//     Hbar_i = <alpha, P_X pi_i> + <beta, nu_i> - eps |nu_i| + eps |mu_i| |nu|
//              + lam KL(P_X pi_i | mu_i)
// (the score of a diagonal-scaling cell plan) are those of the cell plans.
// Everything is evaluated in the log domain in FP64; the cost is separable, so
// each basic cell first forms G(x1, y2) = LSE_{x2} [a(x) - ch (x2 - y2)^2]
// (a = alpha/eps + log mu) for the window's columns and then needs only s
// terms per Y point.
#include "dd_types.h"

#include <limits.h>

namespace dduot {

// ---- interpolation of a potential to the grid with twice the points -------
// Coarse point I stands for the fine points {2I, 2I+1}, i.e. the fine position
// 2I + 1/2; linear between the two nearest centres, continued linearly past
// the first and last ones (a single coarse point: constant).
__device__ __forceinline__ void interp_axis(int i, int nc, int& k, double& t) {
  if (nc == 1) {
    k = 0;
    t = 0.0;
    return;
  }
  const double u = (i - 0.5) * 0.5;
  int kk = (int)floor(u);
  kk = kk < 0 ? 0 : (kk > nc - 2 ? nc - 2 : kk);
  k = kk;
  t = u - kk;
}

__global__ void k_interp(const double* ac, int n1c, int n2c, double* af) {
  const int n1 = 2 * n1c, n2 = 2 * n2c;
  const long n = (long)n1 * n2;
  for (long g = blockIdx.x * (long)blockDim.x + threadIdx.x; g < n; g += (long)gridDim.x * blockDim.x) {
    const int i1 = (int)(g / n2), i2 = (int)(g - (long)i1 * n2);
    int k1, k2;
    double t1, t2;
    interp_axis(i1, n1c, k1, t1);
    interp_axis(i2, n2c, k2, t2);
    const int q1 = n1c == 1 ? 0 : k1 + 1, q2 = n2c == 1 ? 0 : k2 + 1;
    // axis 0 first, then axis 1 (the order of the written-out definition)
    const double lo = (1.0 - t1) * ac[(long)k1 * n2c + k2] + t1 * ac[(long)q1 * n2c + k2];
    const double hi = (1.0 - t1) * ac[(long)k1 * n2c + q2] + t1 * ac[(long)q1 * n2c + q2];
    af[g] = (1.0 - t2) * lo + t2 * hi;
  }
}

hipError_t launch_interp(const double* ac, int n1c, int n2c, double* af, hipStream_t st) {
  const long n = 4L * n1c * n2c;
  const int blocks = (int)((n + 255) / 256 < 4096 ? (n + 255) / 256 : 4096);
  hipLaunchKernelGGL(k_interp, dim3(blocks), dim3(256), 0, st, ac, n1c, n2c, af);
  return hipGetLastError();
}

// ---- basic-cell state from a pair of potentials ----------------------------

constexpr int kMaxS = kMaxTile / 2;

__device__ __forceinline__ void minmax4(int (&v)[4], int* red) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    v[0] = min(v[0], __shfl_xor(v[0], o, 64));
    v[1] = min(v[1], __shfl_xor(v[1], o, 64));
    v[2] = max(v[2], __shfl_xor(v[2], o, 64));
    v[3] = max(v[3], __shfl_xor(v[3], o, 64));
  }
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0)
    for (int k = 0; k < 4; ++k) red[w * 4 + k] = v[k];
  __syncthreads();
  for (int ww = 0; ww < kBlock / 64; ++ww) {
    v[0] = min(v[0], red[ww * 4 + 0]);
    v[1] = min(v[1], red[ww * 4 + 1]);
    v[2] = max(v[2], red[ww * 4 + 2]);
    v[3] = max(v[3], red[ww * 4 + 3]);
  }
  __syncthreads();
}

template <int N>
__device__ __forceinline__ void sumN(double (&v)[N], double* red) {
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

// One workgroup per basic cell.  Dynamic LDS: G (s x gcols) then H (hrows x s).
__global__ __launch_bounds__(kBlock) void k_from_duals(DualsArgs A) {
  extern __shared__ __align__(16) double sm[];
  __shared__ double sa[kMaxS * kMaxS];
  __shared__ double red[4 * (kBlock / 64)];
  __shared__ int redi[4 * (kBlock / 64)];
  const int b = blockIdx.x, t = threadIdx.x, s = A.s;
  const int X1 = A.bxy[b].x, X2 = A.bxy[b].y;
  const Box w = A.win[b];
  double* G = sm;
  double* H = sm + (long)s * A.gcols;
  const double ie = 1.0 / A.eps, ch = A.ch;
  for (int o = t; o < s * s; o += kBlock) {
    const long g = (long)(X1 + o / s) * A.n2 + X2 + o % s;
    sa[o] = A.alpha[g] * ie + log(A.mu[g]);
  }
  __syncthreads();
  // G(x1, y2) = LSE_{x2} [a(x1, x2) - ch (X2 + x2 - y2)^2] over the window columns
  for (int o = t; o < s * w.l2; o += kBlock) {
    const int a1 = o / w.l2, c = o - a1 * w.l2;
    const int y2 = w.o2 + c;
    double m = -INFINITY;
    for (int x2 = 0; x2 < s; ++x2) {
      const double d = (double)(X2 + x2 - y2);
      m = fmax(m, sa[a1 * s + x2] - ch * d * d);
    }
    double acc = 0.0;
    for (int x2 = 0; x2 < s; ++x2) {
      const double d = (double)(X2 + x2 - y2);
      acc += exp(sa[a1 * s + x2] - ch * d * d - m);
    }
    G[a1 * w.l2 + c] = m + log(acc);
  }
  __syncthreads();
  // nu_i(y) = exp(log nu(y) + beta(y)/eps + LSE_{x1} [G(x1, y2) - ch (X1 + x1 - y1)^2])
  auto nu_i = [&](int y1, int y2) -> double {
    const long g = (long)y1 * A.n2 + y2;
    const double* gc = G + (y2 - w.o2);
    double m = -INFINITY;
    for (int x1 = 0; x1 < s; ++x1) {
      const double d = (double)(X1 + x1 - y1);
      m = fmax(m, gc[(long)x1 * w.l2] - ch * d * d);
    }
    double acc = 0.0;
    for (int x1 = 0; x1 < s; ++x1) {
      const double d = (double)(X1 + x1 - y1);
      acc += exp(gc[(long)x1 * w.l2] - ch * d * d - m);
    }
    return exp(log(A.nu[g]) + A.beta[g] * ie + m + log(acc));
  };
  auto kept = [&](double v) { return v >= A.trunc && v > 0.0; };
  // 1. bounding box of the kept points of the window
  if (A.phase == 0) {
    int bb[4] = {INT_MAX, INT_MAX, INT_MIN, INT_MIN};
    for (long o = t; o < (long)w.l1 * w.l2; o += kBlock) {
      const int y1 = w.o1 + (int)(o / w.l2), y2 = w.o2 + (int)(o % w.l2);
      if (kept(nu_i(y1, y2))) {
        bb[0] = min(bb[0], y1);
        bb[1] = min(bb[1], y2);
        bb[2] = max(bb[2], y1 + 1);
        bb[3] = max(bb[3], y2 + 1);
      }
    }
    minmax4(bb, redi);
    Box nb{X1, X2, 0, 0};
    if (bb[0] != INT_MAX) {
      nb.o1 = bb[0];
      nb.o2 = bb[1];
      nb.l1 = bb[2] - bb[0];
      nb.l2 = bb[3] - bb[1];
    }
    if (t == 0) A.box[b] = nb;
    return;
  }
  const Box nb = A.box[b];
  // 2. slot values, <beta, nu_i> and |nu_i|
  double* v = A.vals + A.voff[b];
  double acc2[2] = {0.0, 0.0};
  for (long o = t; o < (long)nb.l1 * nb.l2; o += kBlock) {
    const int y1 = nb.o1 + (int)(o / nb.l2), y2 = nb.o2 + (int)(o % nb.l2);
    const double e = nu_i(y1, y2);
    const double val = kept(e) ? e : 0.0;
    v[o] = val;
    acc2[0] += A.beta[(long)y1 * A.n2 + y2] * val;
    acc2[1] += val;
  }
  sumN<2>(acc2, red);
  __threadfence_block();
  __syncthreads();
  // 3. H(r, x2) = LSE over the kept box points of row r of
  //    log nu(y) + beta(y)/eps - ch (X2 + x2 - y2)^2
  for (int o = t; o < nb.l1 * s; o += kBlock) {
    const int r = o / s, x2 = o - r * s;
    const int y1 = nb.o1 + r;
    const double* vr = v + (long)r * nb.l2;
    double m = -INFINITY;
    for (int c = 0; c < nb.l2; ++c) {
      if (!(vr[c] > 0.0)) continue;
      const long g = (long)y1 * A.n2 + nb.o2 + c;
      const double d = (double)(X2 + x2 - nb.o2 - c);
      m = fmax(m, log(A.nu[g]) + A.beta[g] * ie - ch * d * d);
    }
    double acc = 0.0;
    if (m > -INFINITY)
      for (int c = 0; c < nb.l2; ++c) {
        if (!(vr[c] > 0.0)) continue;
        const long g = (long)y1 * A.n2 + nb.o2 + c;
        const double d = (double)(X2 + x2 - nb.o2 - c);
        acc += exp(log(A.nu[g]) + A.beta[g] * ie - ch * d * d - m);
      }
    H[o] = m > -INFINITY ? m + log(acc) : -INFINITY;
  }
  __syncthreads();
  // 4. P_X pi_i(x) = exp(a(x) + LSE_r [H(r, x2) - ch (X1 + x1 - y1)^2]) and the
  //    x terms of Hbar_i
  double acc3[1] = {0.0};
  for (int o = t; o < s * s; o += kBlock) {
    const int x1 = o / s, x2 = o - x1 * s;
    double m = -INFINITY;
    for (int r = 0; r < nb.l1; ++r) {
      const double d = (double)(X1 + x1 - nb.o1 - r);
      m = fmax(m, H[r * s + x2] - ch * d * d);
    }
    double p = 0.0;
    if (m > -INFINITY) {
      double acc = 0.0;
      for (int r = 0; r < nb.l1; ++r) {
        const double d = (double)(X1 + x1 - nb.o1 - r);
        acc += exp(H[r * s + x2] - ch * d * d - m);
      }
      p = exp(sa[o] + m + log(acc));
    }
    const long g = (long)(X1 + x1) * A.n2 + X2 + x2;
    const double mu = A.mu[g];
    A.px[g] = p;
    const double klx = (p > 0.0 ? p * log(p / mu) : 0.0) - p + mu;
    acc3[0] += A.alpha[g] * p + A.lam * klx + A.eps * mu * A.mass_nu;
  }
  sumN<1>(acc3, red);
  if (t == 0) A.hbar[b] = acc3[0] + acc2[0] - A.eps * acc2[1];
}

size_t from_duals_lds(int s, int gcols, int hrows) {
  return sizeof(double) * ((size_t)s * gcols + (size_t)hrows * s);
}

hipError_t launch_from_duals(const DualsArgs& A, int nbasic, hipStream_t st) {
  if (nbasic <= 0) return hipSuccess;
  const size_t lds = from_duals_lds(A.s, A.gcols, A.hrows);
  hipError_t e = hipFuncSetAttribute((const void*)k_from_duals,
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_from_duals, dim3(nbasic), dim3(kBlock), lds, st, A);
  return hipGetLastError();
}

}  // namespace dduot
