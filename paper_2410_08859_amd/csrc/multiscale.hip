// Coarse-to-fine refinement of a domain-decomposition state (multiscale warm
// start, Sec. 4.4 "Multi-scale and eps-scaling").
//
// A coarse grid has half the points per axis; coarse point X covers the 2 x 2
// fine points x with X = x / 2, and the coarse masses are the sums of the fine
// ones.  The coarse plan pi_c is carried to the fine grid by splitting every
// coarse entry in proportion to the fine masses,
//     pi_f(x, y) = pi_c(X, Y) mu_f(x) / mu_c(X) * nu_f(y) / nu_c(Y),
// which keeps both marginals' shapes inside every coarse point.  The state
// stores basic-cell Y-marginals only; a fine basic cell i lies inside one
// coarse basic cell I, and its Y-marginal is taken as the share
// |mu_f(X_i)| / |mu_c(X_I)| of the refined marginal of I (exact when the
// coarse plan splits X_I proportionally to mu, the only information the stored
// state keeps).  Boxes double; entries below the truncation threshold are
// dropped and the box shrinks to the bounding box of what is left.  Two
// launches: the new boxes (phase 0), then, once the host has placed them in
// the fine state pool, the values (phase 1).
#include "dd_types.h"

#include <limits.h>

namespace dduot {


__device__ __forceinline__ void block_minmax4(int (&v)[4], int* red) {
  // v = {min o1, min o2, max e1, max e2} over the workgroup (256 threads)
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

__device__ __forceinline__ double block_sum1(double x, double* red) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) x += __shfl_down(x, o, 64);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) red[w] = x;
  __syncthreads();
  double s = 0.0;
  for (int ww = 0; ww < kBlock / 64; ++ww) s += red[ww];
  __syncthreads();
  return s;
}

// One workgroup per fine basic cell.
__global__ __launch_bounds__(kBlock) void k_refine_slots(RefineArgs A) {
  __shared__ double redd[kBlock / 64];
  __shared__ int redi[4 * (kBlock / 64)];
  const int b = blockIdx.x;
  const int t = threadIdx.x;
  const int x1 = A.fxy[b].x, x2 = A.fxy[b].y;
  const int X1 = x1 / 2, X2 = x2 / 2;
  const int I = (X1 / A.cs) * A.cnb2 + (X2 / A.cs);
  const int cx1 = (X1 / A.cs) * A.cs, cx2 = (X2 / A.cs) * A.cs;
  // share of the fine basic cell in the coarse basic cell's X mass
  double mf = 0.0, mc = 0.0;
  for (int o = t; o < A.fs * A.fs; o += kBlock) {
    const int a1 = o / A.fs, a2 = o - a1 * A.fs;
    mf += A.mu_f[(long)(x1 + a1) * A.fn2 + (x2 + a2)];
  }
  for (int o = t; o < A.cs * A.cs; o += kBlock) {
    const int a1 = o / A.cs, a2 = o - a1 * A.cs;
    mc += A.mu_c[(long)(cx1 + a1) * A.cn2 + (cx2 + a2)];
  }
  mf = block_sum1(mf, redd);
  mc = block_sum1(mc, redd);
  const double f = mf / mc;
  const Box cb = A.cbox[I];
  const double* cv = A.cvals + A.cvoff[I];
  auto value = [&](int y1, int y2) {
    const int Y1 = y1 / 2, Y2 = y2 / 2;
    return f * cv[(long)(Y1 - cb.o1) * cb.l2 + (Y2 - cb.o2)] * A.nu_f[(long)y1 * A.fn2 + y2] /
           A.nu_c[(long)Y1 * A.cn2 + Y2];
  };
  if (A.phase == 1) {
    const Box nb = A.fbox[b];
    double* fv = A.fvals + A.fvoff[b];
    for (long o = t; o < (long)nb.l1 * nb.l2; o += kBlock) {
      const int a1 = (int)(o / nb.l2), a2 = (int)(o - (long)a1 * nb.l2);
      const double v = value(nb.o1 + a1, nb.o2 + a2);
      fv[o] = v >= A.trunc ? v : 0.0;
    }
    return;
  }
  const int o1 = 2 * cb.o1, o2 = 2 * cb.o2, L1 = 2 * cb.l1, L2 = 2 * cb.l2;
  // bounding box of the refined entries that survive truncation
  int bb[4] = {INT_MAX, INT_MAX, INT_MIN, INT_MIN};
  for (long o = t; o < (long)L1 * L2; o += kBlock) {
    const int a1 = (int)(o / L2), a2 = (int)(o - (long)a1 * L2);
    const int y1 = o1 + a1, y2 = o2 + a2;
    const double v = value(y1, y2);
    if (v >= A.trunc && v > 0.0) {
      bb[0] = min(bb[0], y1);
      bb[1] = min(bb[1], y2);
      bb[2] = max(bb[2], y1 + 1);
      bb[3] = max(bb[3], y2 + 1);
    }
  }
  block_minmax4(bb, redi);
  Box nb{0, 0, 0, 0};
  if (bb[0] != INT_MAX) {
    nb.o1 = bb[0];
    nb.o2 = bb[1];
    nb.l1 = bb[2] - bb[0];
    nb.l2 = bb[3] - bb[1];
  }
  if (t == 0) {
    A.fbox[b] = nb;
    A.fhbar[b] = f * A.chbar[I];
    A.fwarm[b] = A.cwarm[I];
  }
}

// Fine X-marginal from the coarse one.
__global__ void k_refine_grid(const double* px_c, const double* mu_c, const double* mu_f,
                              double* px_f, int fn1, int fn2, int cn2) {
  const long n = (long)fn1 * fn2;
  for (long g = blockIdx.x * (long)blockDim.x + threadIdx.x; g < n; g += (long)gridDim.x * blockDim.x) {
    const int x1 = (int)(g / fn2), x2 = (int)(g - (long)x1 * fn2);
    const long G = (long)(x1 / 2) * cn2 + x2 / 2;
    px_f[g] = px_c[G] * mu_f[g] / mu_c[G];
  }
}

hipError_t launch_interp(const double* ac, int n1c, int n2c, double* af, hipStream_t st);

// Phase 0 (the boxes, hbar, P_X, the stitched potential and its flags) or
// phase 1 (the values at A.fvoff).
hipError_t launch_refine(const RefineArgs& A, int fnbasic, const double* px_c, const double* abar_c,
                         double* px_f, double* abar_f, int fn1, hipStream_t st) {
  if (fnbasic > 0) hipLaunchKernelGGL(k_refine_slots, dim3(fnbasic), dim3(kBlock), 0, st, A);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || A.phase == 1) return e;
  const long n = (long)fn1 * A.fn2;
  const int blocks = (int)((n + 255) / 256 < 8192 ? (n + 255) / 256 : 8192);
  hipLaunchKernelGGL(k_refine_grid, dim3(blocks), dim3(256), 0, st, px_c, A.mu_c, A.mu_f, px_f, fn1,
                     A.fn2, A.cn2);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  // the stored potential (cost units), interpolated linearly: an error of its
  // curvature times h^2 instead of its gradient times h for a block copy
  return launch_interp(abar_c, fn1 / 2, A.fn2 / 2, abar_f, st);
}

}  // namespace dduot
