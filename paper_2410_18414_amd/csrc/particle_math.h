// Per-particle arithmetic shared by the untiled and tiled particle kernels:
// spline weights, periodic wrap, global-memory gather/deposit, IAEM push.
//
// Paper: IAEM (Sec. 4.1); v from the generalized momentum (Sec. 2.2); the
// shape function is a tensor product of centred cardinal B-splines (Sec. 2.2
// and Sec. 4.1 cite it without printing it): nodes at i dx, a particle at
// xi = x/dx touches nodes s .. s+DEG with the per-node weights of Spline::eval.
#pragma once

#include "pic_internal.h"

namespace pic {

template <typename T, int DEG>
struct Spline {
  static constexpr int NW = DEG + 1;
  // eval_unit: the weights times kUnit (cubic: 6 w, its common factor 1/6 left
  // out; other degrees: w), for passes that fold 1 / kUnit^2 into the
  // constants the weight products multiply
  static constexpr double kUnit = DEG == 3 ? 6.0 : 1.0;
  __device__ __forceinline__ static void eval_unit(T xi, int& s, T* w) {
    if constexpr (DEG == 3) {
      const T f = floor(xi);
      const T d = xi - f;  // in [0, 1)
      s = (int)f - 1;
      const T d2 = d * d, d3 = d2 * d, e = T(1) - d;
      w[0] = e * e * e;
      w[1] = T(4) - T(6) * d2 + T(3) * d3;
      w[2] = T(1) + T(3) * d + T(3) * d2 - T(3) * d3;
      w[3] = d3;
    } else {
      eval(xi, s, w);
    }
  }
  // first node index s (may be -1 or up to n+1 before wrapping) and weights
  __device__ __forceinline__ static void eval(T xi, int& s, T* w) {
    if (DEG == 1) {
      const T f = floor(xi);
      const T d = xi - f;
      s = (int)f;
      w[0] = T(1) - d;
      w[1] = d;
    } else if (DEG == 2) {
      const T f = floor(xi + T(0.5));
      const T d = xi - f;  // in [-1/2, 1/2)
      s = (int)f - 1;
      const T a = T(0.5) - d, b = T(0.5) + d;
      w[0] = T(0.5) * a * a;
      w[1] = T(0.75) - d * d;
      w[2] = T(0.5) * b * b;
    } else if (DEG == 3) {
      const T f = floor(xi);
      const T d = xi - f;  // in [0, 1)
      s = (int)f - 1;
      const T d2 = d * d, d3 = d2 * d, e = T(1) - d;
      const T sixth = T(1) / T(6);
      w[0] = e * e * e * sixth;
      w[1] = (T(4) - T(6) * d2 + T(3) * d3) * sixth;
      w[2] = (T(1) + T(3) * d + T(3) * d2 - T(3) * d3) * sixth;
      w[3] = d3 * sixth;
    } else if (DEG == 4) {
      // quartic: nodes round(xi) - 2 .. + 2, w_k = M_4(k - 2 - d) by the
      // pieces of M_4 on |t| < 1/2, 1/2 .. 3/2, 3/2 .. 5/2
      const T f = floor(xi + T(0.5));
      const T d = xi - f;  // in [-1/2, 1/2)
      s = (int)f - 2;
      auto mid = [](T u) {
        const T u2 = u * u;
        return (T(55) + T(20) * u - T(120) * u2 + T(80) * u2 * u - T(16) * u2 * u2) * (T(1) / T(96));
      };
      const T a = T(1) - T(2) * d, b = T(1) + T(2) * d, d2 = d * d;
      w[0] = a * a * a * a * (T(1) / T(384));
      w[1] = mid(T(1) + d);
      w[2] = T(115) / T(192) - T(0.625) * d2 + T(0.25) * d2 * d2;
      w[3] = mid(T(1) - d);
      w[4] = b * b * b * b * (T(1) / T(384));
    } else {
      // quintic: nodes floor(xi) - 2 .. + 3, w_k = M_5(k - 2 - d) by the
      // pieces of M_5 on |t| < 1, 1 .. 2, 2 .. 3
      const T f = floor(xi);
      const T d = xi - f;  // in [0, 1)
      s = (int)f - 2;
      auto inner = [](T u) {
        const T u2 = u * u;
        return T(0.55) - T(0.5) * u2 + T(0.25) * u2 * u2 - u2 * u2 * u * (T(1) / T(12));
      };
      auto mid = [](T u) {
        const T u2 = u * u;
        return T(17) / T(40) + T(0.625) * u - T(1.75) * u2 + T(1.25) * u2 * u - T(0.375) * u2 * u2 +
               u2 * u2 * u * (T(1) / T(24));
      };
      const T e = T(1) - d, e2 = e * e, d2 = d * d;
      w[0] = e2 * e2 * e * (T(1) / T(120));
      w[1] = mid(T(1) + d);
      w[2] = inner(d);
      w[3] = inner(e);
      w[4] = mid(T(2) - d);
      w[5] = d2 * d2 * d * (T(1) / T(120));
    }
  }
  // weights and their derivatives dw/dxi (the adjoint passes differentiate
  // through the particle position)
  __device__ __forceinline__ static void eval_d(T xi, int& s, T* w, T* dw) {
    static_assert(DEG <= 3, "the adjoint passes support spline degrees 1..3");
    eval(xi, s, w);
    if (DEG == 1) {
      dw[0] = T(-1);
      dw[1] = T(1);
    } else if (DEG == 2) {
      const T d = xi - T(s + 1);
      dw[0] = d - T(0.5);
      dw[1] = T(-2) * d;
      dw[2] = d + T(0.5);
    } else {
      const T d = xi - T(s + 1);
      const T e = T(1) - d;
      dw[0] = T(-0.5) * e * e;
      dw[1] = d * (T(1.5) * d - T(2));
      dw[2] = T(0.5) + d - T(1.5) * d * d;
      dw[3] = T(0.5) * d * d;
    }
  }
};

__device__ __forceinline__ int wrapi(int i, int n) { return i < 0 ? i + n : (i >= n ? i - n : i); }

// x in (-L, 2L) -> [0, L); a value that rounds to L is set to 0 (selects,
// not branches: a wave's lanes take different arms)
template <typename T>
__device__ __forceinline__ T wrapx(T x, T L) {
  x = x < T(0) ? x + L : x;
  x = x >= L ? x - L : x;
  return x >= L ? T(0) : x;
}

// node coordinates xi = x/dx, eta = y/dy inside [0, n] (NaN fails the test);
// the stencil of such a point stays within one period of the wrap
template <typename T>
__device__ __forceinline__ bool in_box(T xi, T eta, const GridP& g) {
  // all four tests evaluated (no short-circuit): one branch on the result
  return (xi >= T(0)) & (xi <= T(g.nx)) & (eta >= T(0)) & (eta <= T(g.ny));
}

// deposit with global float64 atomics, stencil already evaluated
template <typename T, int DEG>
__device__ __forceinline__ void deposit_global(int sx, int sy, const T* wx, const T* wy, T jx, T jy, T jz,
                                               double* __restrict__ J, const GridP& g) {
  using S = Spline<T, DEG>;
  const size_t plane = (size_t)g.nx * g.ny;
  const gptr<double> Jg = gp(J);
#pragma unroll
  for (int b = 0; b < S::NW; ++b) {
    const size_t row = (size_t)wrapi(sy + b, g.ny) * g.nx;
#pragma unroll
    for (int a = 0; a < S::NW; ++a) {
      const T w = wx[a] * wy[b];
      const size_t o = row + wrapi(sx + a, g.nx);
      gadd(Jg + o, (double)(jx * w));
      gadd(Jg + plane + o, (double)(jy * w));
      gadd(Jg + 2 * plane + o, (double)(jz * w));
    }
  }
}

// s S(x_g - x) added to one real mesh plane (global float64 atomics)
template <typename T, int DEG>
__device__ __forceinline__ void deposit_scalar_one(T x, T y, T s, double* __restrict__ R, const GridP& g) {
  using S = Spline<T, DEG>;
  const T xi = x * T(g.inv_dx), eta = y * T(g.inv_dy);
  if (!in_box(xi, eta, g)) return;  // non-finite or unwrapped: touch no memory
  int sx, sy;
  T wx[S::NW], wy[S::NW];
  S::eval(xi, sx, wx);
  S::eval(eta, sy, wy);
#pragma unroll
  for (int b = 0; b < S::NW; ++b) {
    const size_t row = (size_t)wrapi(sy + b, g.ny) * g.nx;
#pragma unroll
    for (int a = 0; a < S::NW; ++a) atomicAdd(R + row + wrapi(sx + a, g.nx), (double)(s * wx[a] * wy[b]));
  }
}

template <typename T, int DEG>
__device__ __forceinline__ void deposit_one(T x, T y, T jx, T jy, T jz, double* __restrict__ J,
                                            const GridP& g) {
  using S = Spline<T, DEG>;
  const T xi = x * T(g.inv_dx), eta = y * T(g.inv_dy);
  if (!in_box(xi, eta, g)) return;  // non-finite or unwrapped: touch no memory
  int sx, sy;
  T wx[S::NW], wy[S::NW];
  S::eval(xi, sx, wx);
  S::eval(eta, sy, wy);
  deposit_global<T, DEG>(sx, sy, wx, wy, jx, jy, jz, J, g);
}

// gathered values: 0 dphi/dx, 1 dphi/dy, 2..4 A, 5..7 dA/dx, 8..10 dA/dy,
// read from the planar mesh fields F[f][ny][nx]; out is accumulated into
// Mesh fields read by the gathers: float64 planar, float32 node-major (see
// kFieldSlots)
template <typename T>
__device__ __forceinline__ T field_at(const gptr<const T> F, int f, size_t node, size_t plane) {
  if constexpr (sizeof(T) == 4)
    return F[node * kFieldSlots + f];
  else
    return F[f * plane + node];
}

// The summation order is that of the tiled passes' LDS-window gather (node
// weight wx[a] wy[b], rows outer, columns inner, one multiply-add per field),
// so a particle gathers the same bits from either path: which path it takes
// depends on how far it drifted since the last sort, and the deterministic
// mode's results must not.
template <typename T, int DEG>
__device__ __forceinline__ void gather_global(int sx, int sy, const T* wx, const T* wy, const T* __restrict__ F,
                                              const GridP& g, T* out) {
  using S = Spline<T, DEG>;
  const size_t plane = (size_t)g.nx * g.ny;
  const gptr<const T> Fg = gp(F);
#pragma unroll
  for (int b = 0; b < S::NW; ++b) {
    const size_t row = (size_t)wrapi(sy + b, g.ny) * g.nx;
#pragma unroll
    for (int a = 0; a < S::NW; ++a) {
      const size_t o = row + wrapi(sx + a, g.nx);
      const T w = wx[a] * wy[b];
#pragma unroll
      for (int f = 0; f < 11; ++f) out[f] += w * field_at<T>(Fg, f, o, plane);
    }
  }
}

template <typename T, int DEG>
__device__ __forceinline__ void gather_one(T x, T y, const T* __restrict__ F, const GridP& g, T* out) {
  using S = Spline<T, DEG>;
#pragma unroll
  for (int f = 0; f < 11; ++f) out[f] = T(0);
  const T xi = x * T(g.inv_dx), eta = y * T(g.inv_dy);
  if (!in_box(xi, eta, g)) return;  // non-finite or unwrapped: touch no memory
  int sx, sy;
  T wx[S::NW], wy[S::NW];
  S::eval(xi, sx, wx);
  S::eval(eta, sy, wy);
  gather_global<T, DEG>(sx, sy, wx, wy, F, g, out);
}

// a * b + c, one rounding
__device__ __forceinline__ float fmat(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ __forceinline__ double fmat(double a, double b, double c) { return __builtin_fma(a, b, c); }

// IAEM: v* = 2 v^n - v^{n-1}; P += q dt (-grad phi + (grad A).v*) (x, y only:
// d/dz = 0); v = c^2 u / sqrt(c^2 |u|^2 + (m c^2)^2), u = P - q A.
// A sum of two products can be contracted into a multiply-add either way;
// those sums are written with explicit multiply-adds so that every copy of
// this code the compiler makes rounds the same way (the deterministic mode
// relies on it).
template <typename T>
__device__ __forceinline__ void push_one(const T* gv, T& Px, T& Py, T Pz, T vx, T vy, T vz, T wx, T wy,
                                         T wz, const PhysP& ph, T& nx, T& ny, T& nz) {
  const T q = T(ph.q), dt = T(ph.dt), c = T(ph.c), m = T(ph.m);
  const T sx = T(2) * vx - wx, sy = T(2) * vy - wy, sz = T(2) * vz - wz;
  const T Fx = fmat(sz, gv[7], fmat(sy, gv[6], fmat(sx, gv[5], -gv[0])));
  const T Fy = fmat(sz, gv[10], fmat(sy, gv[9], fmat(sx, gv[8], -gv[1])));
  Px = fmat(q * Fx, dt, Px);
  Py = fmat(q * Fy, dt, Py);
  const T ux = fmat(-q, gv[2], Px), uy = fmat(-q, gv[3], Py), uz = fmat(-q, gv[4], Pz);
  const T c2 = c * c, mc2 = m * c2;
  const T s2 = fmat(c2, fmat(uz, uz, fmat(uy, uy, ux * ux)), mc2 * mc2);
  T inv;
  if constexpr (sizeof(T) == 4)
    inv = c2 * __builtin_amdgcn_rsqf(s2);  // hardware reciprocal square root, about 1 ulp
  else
    inv = c2 / sqrt(s2);
  nx = ux * inv;
  ny = uy * inv;
  nz = uz * inv;
}

// v[t] <- v[(t + r) % NW] for a per-lane r in [0, NW): a barrel shifter, one
// select per element and bit of r, with the lane masks of the bits held in
// scalar registers (written as explicit selects: the compiler otherwise turns
// the shifter back into per-element compare chains)
__device__ __forceinline__ float select_lanes(float a, float b, uint64_t lanes) {
  float r;
  asm("v_cndmask_b32_e64 %0, %1, %2, %3" : "=v"(r) : "v"(a), "v"(b), "s"(lanes));
  return r;
}
__device__ __forceinline__ double select_lanes(double a, double b, uint64_t lanes) {
  const float lo = select_lanes(__uint_as_float((uint32_t)__double_as_longlong(a)),
                                __uint_as_float((uint32_t)__double_as_longlong(b)), lanes);
  const float hi = select_lanes(__uint_as_float((uint32_t)((unsigned long long)__double_as_longlong(a) >> 32)),
                                __uint_as_float((uint32_t)((unsigned long long)__double_as_longlong(b) >> 32)),
                                lanes);
  return __longlong_as_double((long long)(((unsigned long long)__float_as_uint(hi) << 32) | __float_as_uint(lo)));
}
template <int NW, typename T>
__device__ __forceinline__ void rotate_lanes(T (&v)[NW], int r) {
#pragma unroll
  for (int s = 1; s < NW; s <<= 1) {
    const uint64_t lanes = __ballot((r & s) != 0);
    T u[NW];
#pragma unroll
    for (int t = 0; t < NW; ++t) u[t] = select_lanes(v[t], v[(t + s) % NW], lanes);
#pragma unroll
    for (int t = 0; t < NW; ++t) v[t] = u[t];
  }
}

}  // namespace pic
