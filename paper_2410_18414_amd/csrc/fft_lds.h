// Complex helpers, the LDS Stockham FFT and the spectral derivative symbols,
// shared by the field solve (field.hip) and its adjoint (adjoint.hip).
#pragma once

#include "pic_internal.h"

namespace pic {
namespace {

__device__ __forceinline__ double2 cadd(double2 a, double2 b) { return make_double2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ double2 csub(double2 a, double2 b) { return make_double2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ double2 cscale(double2 a, double s) { return make_double2(a.x * s, a.y * s); }
__device__ __forceinline__ double2 cmul(double2 a, double2 b) {
  return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ double2 cconj(double2 a) { return make_double2(a.x, -a.y); }
__device__ __forceinline__ double2 mul_i(double2 a) { return make_double2(-a.y, a.x); }      // i a
__device__ __forceinline__ double2 mul_mi(double2 a) { return make_double2(a.y, -a.x); }     // -i a
__device__ __forceinline__ double2 cdivr(double2 a, double r) { return make_double2(a.x / r, a.y / r); }

// B independent length-N FFTs held in LDS at a[f*N + j], any N >= 2.
// Stockham autosort: radix-4 passes while 4 divides the remaining length, a
// radix-2 pass for a remaining factor 2, then one pass per remaining odd
// prime factor p, in which every output is the p-term sum of its butterfly's
// inputs with the twiddle folded into the DFT factor:
// y_q = sum_m v_m w_N^(m (k N/(p Ns) + q N/p)), k = j mod Ns.
// Ping-pongs between a and b and returns the buffer holding the result.
// tw[t] = exp(-2 pi i t / N), t < N.  INV: exp(+...) (unnormalised inverse).
// All threads of the block must call it; the caller synchronises before.
template <bool INV>
__device__ double2* fft_lds(double2* a, double2* b, int N, int B, const double2* __restrict__ tw) {
  const int tid = threadIdx.x, nth = blockDim.x;
  const bool pow2 = (N & (N - 1)) == 0;
  int Ns = 1;
  while (Ns < N) {
    const int rem = N / Ns;
    int r;
    if ((rem & 3) == 0) {
      r = 4;
      const int q = N >> 2;
      const int stride = N / (4 * Ns);
      const int lq = __ffs(q) - 1;
      for (int t = tid; t < B * q; t += nth) {
        const int f = pow2 ? t >> lq : t / q;
        const int j = t - f * q;
        const double2* in = a + f * N;
        double2* out = b + f * N;
        const int k = j & (Ns - 1);  // Ns is a power of two in the radix-4 and radix-2 passes
        double2 v0 = in[j], v1 = in[j + q], v2 = in[j + 2 * q], v3 = in[j + 3 * q];
        if (k) {
          double2 w1 = tw[k * stride], w2 = tw[2 * k * stride], w3 = tw[3 * k * stride];
          if (INV) { w1 = cconj(w1); w2 = cconj(w2); w3 = cconj(w3); }
          v1 = cmul(v1, w1);
          v2 = cmul(v2, w2);
          v3 = cmul(v3, w3);
        }
        const double2 s02 = cadd(v0, v2), d02 = csub(v0, v2);
        const double2 s13 = cadd(v1, v3), d13 = csub(v1, v3);
        const int d = ((j - k) << 2) + k;
        out[d] = cadd(s02, s13);
        out[d + 2 * Ns] = csub(s02, s13);
        if (INV) {
          out[d + Ns] = cadd(d02, mul_i(d13));
          out[d + 3 * Ns] = cadd(d02, mul_mi(d13));
        } else {
          out[d + Ns] = cadd(d02, mul_mi(d13));
          out[d + 3 * Ns] = cadd(d02, mul_i(d13));
        }
      }
    } else if ((rem & 1) == 0) {
      r = 2;
      const int h = N >> 1;
      const int stride = N / (2 * Ns);
      const int lh = __ffs(h) - 1;
      for (int t = tid; t < B * h; t += nth) {
        const int f = pow2 ? t >> lh : t / h;
        const int j = t - f * h;
        const double2* in = a + f * N;
        double2* out = b + f * N;
        const int k = j & (Ns - 1);
        double2 w = tw[k * stride];
        if (INV) w = cconj(w);
        const double2 v0 = in[j], v1 = cmul(in[j + h], w);
        const int d = ((j - k) << 1) + k;
        out[d] = cadd(v0, v1);
        out[d + Ns] = csub(v0, v1);
      }
    } else {
      // smallest (odd) prime factor of the remaining length
      r = rem;
      for (int p = 3; p * p <= rem; p += 2)
        if (rem % p == 0) {
          r = p;
          break;
        }
      const int q = N / r;             // butterflies per transform
      const int stride = N / (r * Ns);
      for (int t = tid; t < B * N; t += nth) {
        const int f = t / N, o = t - f * N;
        const int k = o % Ns, rest = o / Ns;
        const int qq = rest % r, j = (rest / r) * Ns + k;
        const int e = k * stride + qq * q;  // < N
        const double2* in = a + f * N + j;
        double2 y = in[0];
        int idx = 0;
        for (int m = 1; m < r; ++m) {
          idx += e;
          if (idx >= N) idx -= N;
          const double2 w = INV ? cconj(tw[idx]) : tw[idx];
          y = cadd(y, cmul(in[m * q], w));
        }
        b[f * N + o] = y;
      }
    }
    __syncthreads();
    double2* t = a;
    a = b;
    b = t;
    Ns *= r;
  }
  return a;
}

__device__ __forceinline__ double kx_sym(int kx, const GridP& g) {
  return (2 * kx == g.nx) ? 0.0 : 2.0 * M_PI * kx / g.lx;
}
__device__ __forceinline__ double ky_sym(int ky, const GridP& g) {
  if (2 * ky == g.ny) return 0.0;
  const int m = (2 * ky < g.ny) ? ky : ky - g.ny;
  return 2.0 * M_PI * m / g.ly;
}

}  // namespace
}  // namespace pic
