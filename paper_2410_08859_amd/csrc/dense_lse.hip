// Global log-sum-exp over explicit point pairs, FP64, with exact pruning.
//
//   out(o) = log sum_k exp(v_k - ch |p_o - q_k|^2)
//
// for outputs p_o and inputs q_k on two n1 x n2 point sets given in pixel
// units as grid index + displacement (displacement NULL: the grid itself).
// This is the certificate's global Y-update (eq. sinkhorn-iters-ot with
// nu_- = 0) and X-marginal when the Y points are moved and the cost is no
// longer separable, and the first moments sum_x pi(x, y) x of the plan for the
// gradient with respect to the Y positions.
//
// The inputs are grouped in 16 x 16 index blocks with their maximal value and
// the bounding box of their positions, so ub_k = vmax_k - ch dist^2(p, box_k)
// bounds every term of block k.  Per output: the block of largest bound is
// summed exactly first, giving a lower bound L of the result; then every
// block with ub_k >= L - T is summed (relative to a running maximum of its
// terms), T = 37 + log(256 * blocks), so the skipped blocks hold less than
// e^-37 of the result together (below FP64 rounding).  One workgroup covers a 16 x 16 block of outputs; a block is
// staged in LDS when any output of the workgroup needs it.
#include "dd_types.h"

namespace dduot {

constexpr int kB = 16;   // block side

__device__ __forceinline__ double pos_of(const double* del, long g, int ax, int idx) {
  return del ? idx + del[2 * g + ax] : (double)idx;
}

// Per input block: vmax, min/max of both position coordinates.
__global__ __launch_bounds__(kBlock) void k_block_info(const double* v, const double* del, int n1,
                                                        int n2, double* info) {
  __shared__ double red[5 * (kBlock / 64)];
  const int nb2 = (n2 + kB - 1) / kB;
  const int b1 = blockIdx.x / nb2, b2 = blockIdx.x % nb2;
  const int a1 = threadIdx.x / kB, a2 = threadIdx.x % kB;
  const int i1 = b1 * kB + a1, i2 = b2 * kB + a2;
  double m[5] = {-INFINITY, INFINITY, -INFINITY, INFINITY, -INFINITY};
  if (i1 < n1 && i2 < n2) {
    const long g = (long)i1 * n2 + i2;
    const double q1 = pos_of(del, g, 0, i1), q2 = pos_of(del, g, 1, i2);
    m[0] = v[g];
    m[1] = q1; m[2] = q1;
    m[3] = q2; m[4] = q2;
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    m[0] = fmax(m[0], __shfl_xor(m[0], o, 64));
    m[1] = fmin(m[1], __shfl_xor(m[1], o, 64));
    m[2] = fmax(m[2], __shfl_xor(m[2], o, 64));
    m[3] = fmin(m[3], __shfl_xor(m[3], o, 64));
    m[4] = fmax(m[4], __shfl_xor(m[4], o, 64));
  }
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  if (lane == 0)
    for (int k = 0; k < 5; ++k) red[w * 5 + k] = m[k];
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int ww = 1; ww < kBlock / 64; ++ww) {
      m[0] = fmax(m[0], red[ww * 5 + 0]);
      m[1] = fmin(m[1], red[ww * 5 + 1]);
      m[2] = fmax(m[2], red[ww * 5 + 2]);
      m[3] = fmin(m[3], red[ww * 5 + 3]);
      m[4] = fmax(m[4], red[ww * 5 + 4]);
    }
    for (int k = 0; k < 5; ++k) info[5 * (long)blockIdx.x + k] = m[k];
  }
}

__device__ __forceinline__ double block_bound(const double* inf, double p1, double p2, double ch) {
  const double d1 = fmax(fmax(inf[1] - p1, p1 - inf[2]), 0.0);
  const double d2 = fmax(fmax(inf[3] - p2, p2 - inf[4]), 0.0);
  return inf[0] - ch * (d1 * d1 + d2 * d2);
}

// Outputs: o = 16 x 16 block of the output grid per workgroup.  mom (nullable):
// the normalised first moments sum e^t q / sum e^t, 2 per output.
__global__ __launch_bounds__(kBlock) void k_dense_lse(const double* v, const double* qdel,
                                                      const double* info, int n1, int n2,
                                                      const double* pdel, double ch, double* out,
                                                      double* mom) {
  __shared__ double sv[kB * kB], sq1[kB * kB], sq2[kB * kB];
  __shared__ double sinf[5];
  const int nb1 = (n1 + kB - 1) / kB, nb2 = (n2 + kB - 1) / kB, nbk = nb1 * nb2;
  const int ob1 = blockIdx.x / nb2, ob2 = blockIdx.x % nb2;
  const int i1 = ob1 * kB + threadIdx.x / kB, i2 = ob2 * kB + threadIdx.x % kB;
  const bool act = i1 < n1 && i2 < n2;
  const long go = act ? (long)i1 * n2 + i2 : 0;
  const double p1 = act ? pos_of(pdel, go, 0, i1) : 0.0, p2 = act ? pos_of(pdel, go, 1, i2) : 0.0;
  // 1. block of largest bound
  double best = -INFINITY;
  int kbest = 0;
  for (int k = 0; k < nbk; ++k) {
    const double ub = block_bound(info + 5 * (long)k, p1, p2, ch);
    if (ub > best) {
      best = ub;
      kbest = k;
    }
  }
  // 2. lower bound L: exact sum of that block (two passes)
  auto block_terms = [&](int k, double shift, double& s0, double& s1, double& s2, double& mx) {
    const int b1 = k / nb2, b2 = k % nb2;
    for (int a = 0; a < kB * kB; ++a) {
      const int q1i = b1 * kB + a / kB, q2i = b2 * kB + a % kB;
      if (q1i >= n1 || q2i >= n2) continue;
      const long g = (long)q1i * n2 + q2i;
      const double q1 = pos_of(qdel, g, 0, q1i), q2 = pos_of(qdel, g, 1, q2i);
      const double e1 = p1 - q1, e2 = p2 - q2;
      const double t = v[g] - ch * (e1 * e1 + e2 * e2);
      if (shift == -INFINITY) {
        mx = fmax(mx, t);
      } else {
        const double e = exp(t - shift);
        s0 += e;
        s1 += e * q1;
        s2 += e * q2;
      }
    }
  };
  double L = -INFINITY;
  if (act && best > -INFINITY) {
    double s0 = 0, s1 = 0, s2 = 0, mx = -INFINITY;
    block_terms(kbest, -INFINITY, s0, s1, s2, mx);
    if (mx > -INFINITY) {
      block_terms(kbest, mx, s0, s1, s2, mx);
      L = mx + log(s0);
    }
  }
  // 3. every block that can matter, staged in LDS.  The terms are summed
  // relative to a running maximum m (starting at L): a block's actual terms
  // may lie far below its bound, so another block's terms can exceed L by
  // more than exp's range.
  const double T = 37.0 + log(256.0 * nbk);
  double s0 = 0, s1 = 0, s2 = 0, m = L;
  for (int k = 0; k < nbk; ++k) {
    if (threadIdx.x < 5) sinf[threadIdx.x] = info[5 * (long)k + threadIdx.x];
    __syncthreads();
    const bool need = act && L > -INFINITY && block_bound(sinf, p1, p2, ch) >= L - T;
    if (__syncthreads_or(need)) {
      const int b1 = k / nb2, b2 = k % nb2;
      const int a1 = threadIdx.x / kB, a2 = threadIdx.x % kB;
      const int q1i = b1 * kB + a1, q2i = b2 * kB + a2;
      if (q1i < n1 && q2i < n2) {
        const long g = (long)q1i * n2 + q2i;
        sv[threadIdx.x] = v[g];
        sq1[threadIdx.x] = pos_of(qdel, g, 0, q1i);
        sq2[threadIdx.x] = pos_of(qdel, g, 1, q2i);
      } else {
        sv[threadIdx.x] = -INFINITY;
        sq1[threadIdx.x] = 0.0;
        sq2[threadIdx.x] = 0.0;
      }
      __syncthreads();
      if (need) {
        for (int a = 0; a < kB * kB; ++a) {
          const double e1 = p1 - sq1[a], e2 = p2 - sq2[a];
          const double t = sv[a] - ch * (e1 * e1 + e2 * e2);
          if (t > m) {
            const double r = exp(m - t);
            s0 *= r;
            s1 *= r;
            s2 *= r;
            m = t;
          }
          const double e = exp(t - m);
          s0 += e;
          s1 += e * sq1[a];
          s2 += e * sq2[a];
        }
      }
    }
    __syncthreads();
  }
  if (act) {
    out[go] = L > -INFINITY ? m + log(s0) : -INFINITY;
    if (mom) {
      mom[2 * go] = s0 > 0.0 ? s1 / s0 : 0.0;
      mom[2 * go + 1] = s0 > 0.0 ? s2 / s0 : 0.0;
    }
  }
}

// out = LSE over the q points; info: scratch of 5 doubles per input block.
hipError_t dense_lse(const double* v, const double* qdel, const double* pdel, int n1, int n2,
                     double ch, double* info, double* out, double* mom, hipStream_t st) {
  const int nbk = ((n1 + kB - 1) / kB) * ((n2 + kB - 1) / kB);
  hipLaunchKernelGGL(k_block_info, dim3(nbk), dim3(kBlock), 0, st, v, qdel, n1, n2, info);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_dense_lse, dim3(nbk), dim3(kBlock), 0, st, v, qdel, info, n1, n2, pdel, ch,
                     out, mom);
  return hipGetLastError();
}

}  // namespace dduot
