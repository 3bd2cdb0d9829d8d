// Particle kernels: position update + current deposit, gather + IAEM push,
// the fused gather/push/position/deposit pass, and particle state I/O.
//
// Paper: IAEM (Sec. 4.1) and Algorithm 1 (Sec. 4.2); current deposition with
// tensor-product B-splines at x^{n+1} weighted by q v^n (Sec. 4.1: the
// positions place the weights, the old velocities carry the value), full
// order in every direction; the velocity from the generalized momentum
// (Sec. 2.2).
//
// Spline (the paper cites it without printing it): nodes at i dx, centred
// cardinal B-spline of degree DEG; a particle at xi = x/dx touches nodes
// s .. s+DEG with the per-node weights of Spline::eval (particle_math.h).
#include <algorithm>

#include "particle_math.h"

namespace pic {

namespace {

// Untiled passes (PIC_FLAG_NO_SORT, and the naive charge deposit): one
// particle per thread, gather from the mesh fields in global memory (float64
// planar, float32 node-major), deposit with global float64 atomics.
// Flattened over instances (BK_PART blocks of 256 particles each).
template <typename T, int DEG, int MODE>
__global__ void __launch_bounds__(256) k_untiled(const InstDesc* __restrict__ D, int ninst, StepArgs sa) {
  const int ii = find_inst(D, ninst, BK_PART, blockIdx.x);
  const InstDesc& d = D[ii];
  const int64_t i = (int64_t)(blockIdx.x - d.blk[BK_PART]) * 256 + threadIdx.x;
  if (i >= d.n) return;
  const GridP g = d.g;
  const PhysP ph = d.ph;
  const Parts<T> p = make_parts<T>(d, sa.cur, sa.vflip);
  double* __restrict__ J = d.J;
  const T dt = T(ph.dt), q = T(ph.q);
  T x = p.x[i], y = p.y[i];
  T vx = p.v[0][i], vy = p.v[1][i], vz = p.v[2][i];
  // the velocity one level older than the deposited one (v* = 2 v - u in J)
  T ux = T(0), uy = T(0), uz = T(0);
  if (MODE == 0 && d.jvstar) {
    ux = p.w[0][i];
    uy = p.w[1][i];
    uz = p.w[2][i];
  }
  if (MODE != 0) {
    const T* __restrict__ F = d.F32 ? (const T*)(const void*)d.F32 : (const T*)(const void*)d.F64;
    T gv[11];
    gather_one<T, DEG>(x, y, F, g, gv);
    T Px = p.P[0][i], Py = p.P[1][i];
    const T Pz = p.P[2][i];
    const T wx = p.w[0][i], wy = p.w[1][i], wz = p.w[2][i];
    T nx, ny, nz;
    push_one<T>(gv, Px, Py, Pz, vx, vy, vz, wx, wy, wz, ph, nx, ny, nz);
    p.P[0][i] = Px;
    p.P[1][i] = Py;
    p.w[0][i] = nx;
    p.w[1][i] = ny;
    p.w[2][i] = nz;
    ux = vx;
    uy = vy;
    uz = vz;
    vx = nx;
    vy = ny;
    vz = nz;
  }
  if (MODE != 1) {  // position update and deposit with the newest velocity
    if (MODE == 0 && sa.stage >= 0) {
      // sub-stepped DIRK stage: deposit at x + c_i dt v into J planes
      // 3i..3i+2; only the last stage writes x^{n+1}
      if (sa.stage == d.sc.stages - 1) {
        p.x[i] = wrapx<T>(x + vx * dt, T(g.lx));
        p.y[i] = wrapx<T>(y + vy * dt, T(g.ly));
      }
      const T sdt = T(ph.dt * d.sc.dirkC[sa.stage]);
      x = wrapx<T>(x + vx * sdt, T(g.lx));
      y = wrapx<T>(y + vy * sdt, T(g.ly));
      J += (size_t)3 * sa.stage * g.nx * g.ny;
    } else {
      x = wrapx<T>(x + vx * dt, T(g.lx));
      y = wrapx<T>(y + vy * dt, T(g.ly));
      p.x[i] = x;
      p.y[i] = y;
    }
    const T s = q * T(g.inv_area);
    if (d.jvstar) deposit_one<T, DEG>(x, y, s * (T(2) * vx - ux), s * (T(2) * vy - uy), s * (T(2) * vz - uz), J, g);
    else deposit_one<T, DEG>(x, y, s * vx, s * vy, s * vz, J, g);
    // naive comparison: rho^{n+1} from the same spline at x^{n+1}
    if (d.naive) deposit_scalar_one<T, DEG>(x, y, s, J + 3 * (size_t)g.nx * g.ny, g);
  }
}

// s S(x_g - x_p) of every particle added to the plane R (the naive mode's ion
// background: s = -q / (dx dy) at the initial positions)
template <typename T, int DEG>
__global__ void __launch_bounds__(256) k_charge(Parts<T> p, int64_t n, GridP g, double s, double* __restrict__ R) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  deposit_scalar_one<T, DEG>(p.x[i], p.y[i], T(s), R, g);
}

template <typename T>
__global__ void k_init_particles(Parts<T> p, int64_t n, const double* __restrict__ x,
                                 const double* __restrict__ y, const double* __restrict__ P, GridP g,
                                 PhysP ph) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= n) return;
  double xx = x[i] - g.lx * floor(x[i] / g.lx);
  if (xx >= g.lx) xx = 0.0;
  double yy = y[i] - g.ly * floor(y[i] / g.ly);
  if (yy >= g.ly) yy = 0.0;
  const double px = P[i], py = P[n + i], pz = P[2 * n + i];
  const double c2 = ph.c * ph.c, mc2 = ph.m * c2;
  const double inv = c2 / sqrt(c2 * (px * px + py * py + pz * pz) + mc2 * mc2);
  T xt = (T)xx, yt = (T)yy;
  if (xt >= T(g.lx)) xt = T(0);  // rounding to the particle dtype can reach L
  if (yt >= T(g.ly)) yt = T(0);
  p.x[i] = xt;
  p.y[i] = yt;
  p.P[0][i] = (T)px;
  p.P[1][i] = (T)py;
  p.P[2][i] = (T)pz;
  p.v[0][i] = p.w[0][i] = (T)(px * inv);
  p.v[1][i] = p.w[1][i] = (T)(py * inv);
  p.v[2][i] = p.w[2][i] = (T)(pz * inv);
  p.id[i] = (int32_t)i;
}

template <typename T>
__global__ void k_get_particles(Parts<T> p, int64_t n, double* __restrict__ out) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int64_t o = p.id[i];
  const T* src[11] = {p.x, p.y, p.P[0], p.P[1], p.P[2], p.v[0], p.v[1], p.v[2], p.w[0], p.w[1], p.w[2]};
#pragma unroll
  for (int k = 0; k < 11; ++k) out[k * n + o] = (double)src[k][i];
}

template <typename T>
__global__ void k_set_particles(Parts<T> p, int64_t n, const double* __restrict__ in, GridP g) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= n) return;
  T* dst[11] = {p.x, p.y, p.P[0], p.P[1], p.P[2], p.v[0], p.v[1], p.v[2], p.w[0], p.w[1], p.w[2]};
#pragma unroll
  for (int k = 2; k < 11; ++k) dst[k][i] = (T)in[k * n + i];
  double xx = in[i] - g.lx * floor(in[i] / g.lx);
  if (xx >= g.lx) xx = 0.0;
  double yy = in[n + i] - g.ly * floor(in[n + i] / g.ly);
  if (yy >= g.ly) yy = 0.0;
  T xt = (T)xx, yt = (T)yy;
  if (xt >= T(g.lx)) xt = T(0);  // rounding to the particle dtype can reach L
  if (yt >= T(g.ly)) yt = T(0);
  p.x[i] = xt;
  p.y[i] = yt;
  p.id[i] = (int32_t)i;
}

// kinetic energy sum (gamma - 1) m c^2 from v^n, and a count of non-finite
// values; per-block partials in out2[2*block + {0,1}]
template <typename T>
__global__ void __launch_bounds__(256) k_particle_diag(Parts<T> p, int64_t n, PhysP ph, double* out2) {
  __shared__ double s0[256], s1[256];
  double ke = 0, bad = 0;
  const double c2 = ph.c * ph.c;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const T* src[11] = {p.x, p.y, p.P[0], p.P[1], p.P[2], p.v[0], p.v[1], p.v[2], p.w[0], p.w[1], p.w[2]};
    bool fin = true;
#pragma unroll
    for (int k = 0; k < 11; ++k) fin = fin && isfinite((double)src[k][i]);
    if (!fin) {
      bad += 1;
      continue;
    }
    const double vx = p.v[0][i], vy = p.v[1][i], vz = p.v[2][i];
    const double b2 = (vx * vx + vy * vy + vz * vz) / c2;
    ke += (1.0 / sqrt(1.0 - b2) - 1.0) * ph.m * c2;
  }
  s0[threadIdx.x] = ke;
  s1[threadIdx.x] = bad;
  __syncthreads();
  for (int s = blockDim.x / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) {
      s0[threadIdx.x] += s0[threadIdx.x + s];
      s1[threadIdx.x] += s1[threadIdx.x + s];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    out2[2 * blockIdx.x] = s0[0];
    out2[2 * blockIdx.x + 1] = s1[0];
  }
}

__global__ void k_fill_f64(double* p, size_t n, double v) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
    p[i] = v;
}

inline unsigned blocks_for(int64_t n) { return (unsigned)((n + 255) / 256); }

}  // namespace

hipError_t launch_fill_f64(double* p, size_t n, double v, hipStream_t s) {
  const int blocks = (int)std::min<size_t>((n + 255) / 256, 8192);
  if (n) hipLaunchKernelGGL(k_fill_f64, dim3(blocks), dim3(256), 0, s, p, n, v);
  return hipGetLastError();
}

hipError_t launch_charge(int dtype, int degree, const void* parts, int64_t n, GridP g, double s, double* R,
                         hipStream_t st) {
  if (n == 0) return hipSuccess;
  const dim3 nb(blocks_for(n)), th(256);
  if (dtype == PIC_F32) {
    const Parts<float>& p = *(const Parts<float>*)parts;
    if (degree == 1) hipLaunchKernelGGL((k_charge<float, 1>), nb, th, 0, st, p, n, g, s, R);
    else if (degree == 2) hipLaunchKernelGGL((k_charge<float, 2>), nb, th, 0, st, p, n, g, s, R);
    else if (degree == 4) hipLaunchKernelGGL((k_charge<float, 4>), nb, th, 0, st, p, n, g, s, R);
    else if (degree == 5) hipLaunchKernelGGL((k_charge<float, 5>), nb, th, 0, st, p, n, g, s, R);
    else hipLaunchKernelGGL((k_charge<float, 3>), nb, th, 0, st, p, n, g, s, R);
  } else {
    const Parts<double>& p = *(const Parts<double>*)parts;
    if (degree == 1) hipLaunchKernelGGL((k_charge<double, 1>), nb, th, 0, st, p, n, g, s, R);
    else if (degree == 2) hipLaunchKernelGGL((k_charge<double, 2>), nb, th, 0, st, p, n, g, s, R);
    else if (degree == 4) hipLaunchKernelGGL((k_charge<double, 4>), nb, th, 0, st, p, n, g, s, R);
    else if (degree == 5) hipLaunchKernelGGL((k_charge<double, 5>), nb, th, 0, st, p, n, g, s, R);
    else hipLaunchKernelGGL((k_charge<double, 3>), nb, th, 0, st, p, n, g, s, R);
  }
  return hipGetLastError();
}

hipError_t launch_init_particles(int dtype, const void* parts, int64_t n, const double* x, const double* y,
                                 const double* P, GridP g, PhysP ph, hipStream_t s) {
  if (n == 0) return hipSuccess;
  if (dtype == PIC_F32)
    hipLaunchKernelGGL(k_init_particles<float>, dim3(blocks_for(n)), dim3(256), 0, s,
                       *(const Parts<float>*)parts, n, x, y, P, g, ph);
  else
    hipLaunchKernelGGL(k_init_particles<double>, dim3(blocks_for(n)), dim3(256), 0, s,
                       *(const Parts<double>*)parts, n, x, y, P, g, ph);
  return hipGetLastError();
}

template <typename T, int MODE>
static hipError_t launch_untiled_deg(int degree, const InstDesc* D, int ninst, int nblocks, StepArgs sa,
                                     hipStream_t s) {
  switch (degree) {
    case 1: hipLaunchKernelGGL((k_untiled<T, 1, MODE>), dim3(nblocks), dim3(256), 0, s, D, ninst, sa); break;
    case 2: hipLaunchKernelGGL((k_untiled<T, 2, MODE>), dim3(nblocks), dim3(256), 0, s, D, ninst, sa); break;
    case 4: hipLaunchKernelGGL((k_untiled<T, 4, MODE>), dim3(nblocks), dim3(256), 0, s, D, ninst, sa); break;
    case 5: hipLaunchKernelGGL((k_untiled<T, 5, MODE>), dim3(nblocks), dim3(256), 0, s, D, ninst, sa); break;
    default: hipLaunchKernelGGL((k_untiled<T, 3, MODE>), dim3(nblocks), dim3(256), 0, s, D, ninst, sa); break;
  }
  return hipGetLastError();
}

template <typename T>
static hipError_t launch_untiled_mode(int mode, int degree, const InstDesc* D, int ninst, int nblocks, StepArgs sa,
                                      hipStream_t s) {
  switch (mode) {
    case 0: return launch_untiled_deg<T, 0>(degree, D, ninst, nblocks, sa, s);
    case 1: return launch_untiled_deg<T, 1>(degree, D, ninst, nblocks, sa, s);
    default: return launch_untiled_deg<T, 2>(degree, D, ninst, nblocks, sa, s);
  }
}

hipError_t launch_untiled(int dtype, int mode, int degree, const InstDesc* D, int ninst, int nblocks, StepArgs sa,
                          hipStream_t s) {
  if (nblocks == 0) return hipSuccess;
  if (dtype == PIC_F32) return launch_untiled_mode<float>(mode, degree, D, ninst, nblocks, sa, s);
  return launch_untiled_mode<double>(mode, degree, D, ninst, nblocks, sa, s);
}

// largest in-plane velocity component max(|v_x|, |v_y|) of the set, as the
// bits of a non-negative float (which order like the float); a non-finite
// velocity counts as +inf
template <typename T>
__global__ void __launch_bounds__(256) k_max_inplane(Parts<T> p, int64_t n, uint32_t* __restrict__ out) {
  __shared__ float red[256];
  float m = 0.0f;
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
    const float a = fmaxf(fabsf((float)p.v[0][i]), fabsf((float)p.v[1][i]));
    m = a == a ? fmaxf(m, a) : __int_as_float(0x7f800000);
  }
  red[threadIdx.x] = m;
  __syncthreads();
  for (int st = 128; st > 0; st >>= 1) {
    if ((int)threadIdx.x < st) red[threadIdx.x] = fmaxf(red[threadIdx.x], red[threadIdx.x + st]);
    __syncthreads();
  }
  if (threadIdx.x == 0) atomicMax(out, __float_as_uint(red[0]));
}

hipError_t launch_max_inplane(int dtype, const void* parts, int64_t n, uint32_t* out, hipStream_t s) {
  if (n == 0) return hipSuccess;
  const int blocks = (int)std::min<int64_t>(1024, (n + 255) / 256);
  if (dtype == PIC_F32)
    hipLaunchKernelGGL(k_max_inplane<float>, dim3(blocks), dim3(256), 0, s, *(const Parts<float>*)parts, n, out);
  else
    hipLaunchKernelGGL(k_max_inplane<double>, dim3(blocks), dim3(256), 0, s, *(const Parts<double>*)parts, n, out);
  return hipGetLastError();
}

hipError_t launch_get_particles(int dtype, const void* parts, int64_t n, double* out, hipStream_t s) {
  if (n == 0) return hipSuccess;
  if (dtype == PIC_F32)
    hipLaunchKernelGGL(k_get_particles<float>, dim3(blocks_for(n)), dim3(256), 0, s,
                       *(const Parts<float>*)parts, n, out);
  else
    hipLaunchKernelGGL(k_get_particles<double>, dim3(blocks_for(n)), dim3(256), 0, s,
                       *(const Parts<double>*)parts, n, out);
  return hipGetLastError();
}

hipError_t launch_set_particles(int dtype, const void* parts, int64_t n, const double* in, GridP g, hipStream_t s) {
  if (n == 0) return hipSuccess;
  if (dtype == PIC_F32)
    hipLaunchKernelGGL(k_set_particles<float>, dim3(blocks_for(n)), dim3(256), 0, s, *(const Parts<float>*)parts, n,
                       in, g);
  else
    hipLaunchKernelGGL(k_set_particles<double>, dim3(blocks_for(n)), dim3(256), 0, s, *(const Parts<double>*)parts, n,
                       in, g);
  return hipGetLastError();
}

hipError_t launch_particle_diag(int dtype, const void* parts, int64_t n, PhysP ph, double* out2, hipStream_t s) {
  if (dtype == PIC_F32)
    hipLaunchKernelGGL(k_particle_diag<float>, dim3(256), dim3(256), 0, s, *(const Parts<float>*)parts, n, ph,
                       out2);
  else
    hipLaunchKernelGGL(k_particle_diag<double>, dim3(256), dim3(256), 0, s, *(const Parts<double>*)parts, n, ph,
                       out2);
  return hipGetLastError();
}

}  // namespace pic
