// Discrete adjoint of one BDF-k step (Algorithm 1 with the BDF-k update of
// Sec. 3.2), float64, one instance.  Given the step's recomputed forward
// quantities and the adjoint lambda^{n+1} of its outputs, these kernels form
// lambda^n = (d S^{n+1} / d S^n)^T lambda^{n+1}; the state S^n is the particle
// arrays (x, y, P, v^n, v^{n-1}) and the spectral history.
//
// The sweep runs the forward phases backwards:
//   k_adj_push(_t) push and gather adjoint: v' = c^2 u / s (Sec. 2.2) has the
//                  symmetric Jacobian (c^2/s)(I - c^2 u u^T / s^2); the IAEM
//                  force (Sec. 4.1) is linear in the gathered values; the
//                  gather's adjoint scatters lambda_g onto the 11 mesh fields
//                  with the same spline weights and gives lambda_x through the
//                  spline derivative.
//   k_rows_r2c(adj), k_adj_columns, k_rows_c2r(adj)
//                  field-solve adjoint: the real-to-complex transforms of the
//                  11 mesh-field adjoints, the conjugate spectral symbols, the
//                  transposed per-mode BDF recurrence (continuity, both
//                  Helmholtz solves and the history shift), then the adjoint
//                  of J^ = rfft2(J), which is N irfft2(lambda_J^ / w).
//   k_adj_deposit(_t) deposit adjoint: a gather of lambda_J with the spline
//                  weights (lambda_v) and their derivatives (lambda_x), then
//                  the position update x' = x + v dt.
//
// Complex adjoints follow the real-pair convention lambda_z = dL/dRe z + i
// dL/dIm z, so a complex-linear map y = s z transposes to lambda_z = conj(s)
// lambda_y.  For a real field F = irfft2(Z) the adjoint is lambda_Z =
// (w_kx / N) rfft2(lambda_F) with w = 1 on the kx = 0 and kx = nx/2 columns
// and 2 elsewhere.
//
// Adjoint particle state LAM[11][ls] in the slot order of the particle set
// the step runs on (so every access coalesces): x, y, Px, Py, Pz, v^n (3),
// v^{n-1} (3).  LIDS[i] names the original particle held in slot i; when a
// sort changes the set's order, k_lam_* permute LAM to the new one.  Callers
// exchange it in original order (k_lam_set / k_lam_get).
#include "fft_lds.h"
#include "particle_math.h"

#include <algorithm>

namespace pic {

namespace {

// one particle's adjoint: slot k of the arrays at b (wave-uniform base), f * ls apart
struct LamRef {
  gptr<double> b;
  int64_t ls;
  uint32_t k;
  __device__ __forceinline__ __attribute__((address_space(1))) double& operator()(int f) const {
    return elt(b + f * ls, k);
  }
};

// Push adjoint of one particle: gathered values gv at x^{n+1}; P^n, v^n,
// v^{n-1}; lambda^{n+1} in lam in, lambda of P, v^n and v^{n-1} out.  Returns
// lambda_g in lg[11]: the callers scatter it onto the mesh fields and add the
// gather's position term, sum_f lg[f] d gv[f] / dx, to lambda_x (and the same
// for y).
__device__ __forceinline__ void adj_push_one(const double* gv, double P0, double P1, double P2, double v0, double v1,
                                             double v2, double w0, double w1, double w2, const PhysP& ph,
                                             const LamRef& lam, double* lg) {
  // forward push (IAEM) with its intermediates
  const double q = ph.q, dt = ph.dt, c2 = ph.c * ph.c, mc2 = ph.m * c2;
  const double s0 = 2.0 * v0 - w0, s1 = 2.0 * v1 - w1, s2 = 2.0 * v2 - w2;
  const double Fx = -gv[0] + s0 * gv[5] + s1 * gv[6] + s2 * gv[7];
  const double Fy = -gv[1] + s0 * gv[8] + s1 * gv[9] + s2 * gv[10];
  const double ux = P0 + q * Fx * dt - q * gv[2];
  const double uy = P1 + q * Fy * dt - q * gv[3];
  const double uz = P2 - q * gv[4];
  const double ss = sqrt(c2 * (ux * ux + uy * uy + uz * uz) + mc2 * mc2);
  // adjoint of v' = c^2 u / ss
  const double lvx = lam(5), lvy = lam(6), lvz = lam(7);
  const double ud = (ux * lvx + uy * lvy + uz * lvz) * c2 / (ss * ss);
  const double k1 = c2 / ss;
  const double lux = k1 * (lvx - ud * ux), luy = k1 * (lvy - ud * uy), luz = k1 * (lvz - ud * uz);
  // P' = P + q dt (Fx, Fy, 0), u = P' - q A
  const double lPx = lam(2) + lux, lPy = lam(3) + luy, lPz = lam(4) + luz;
  const double lFx = q * dt * lPx, lFy = q * dt * lPy;
  lg[0] = -lFx;
  lg[1] = -lFy;
  lg[2] = -q * lux;
  lg[3] = -q * luy;
  lg[4] = -q * luz;
  lg[5] = lFx * s0;
  lg[6] = lFx * s1;
  lg[7] = lFx * s2;
  lg[8] = lFy * s0;
  lg[9] = lFy * s1;
  lg[10] = lFy * s2;
  // v* = 2 v^n - v^{n-1}
  const double lsx = lFx * gv[5] + lFy * gv[8];
  const double lsy = lFx * gv[6] + lFy * gv[9];
  const double lsz = lFx * gv[7] + lFy * gv[10];
  lam(2) = lPx;  // final: P enters only through P'
  lam(3) = lPy;
  lam(4) = lPz;
  // v^n: the outgoing v^{n-1} slot of S^{n+1} is v^n itself, plus 2 lambda_v*
  lam(5) = lam(8) + 2.0 * lsx;
  lam(6) = lam(9) + 2.0 * lsy;
  lam(7) = lam(10) + 2.0 * lsz;
  lam(8) = -lsx;
  lam(9) = -lsy;
  lam(10) = -lsz;
}

// gathered values and their node-coordinate derivatives from planar fields
// F[f * stride + node] with nodes (sx + a, sy + b) at row pitch `pitch` (a
// window, or the global mesh with wrapped indices when `wrap`)
template <int DEG, int NF, typename Ptr>
__device__ __forceinline__ void gather_d(Ptr F, size_t stride, const double* wx,
                                         const double* dwx, const double* wy, const double* dwy, int sx, int sy,
                                         const GridP& g, int pitch, bool wrap, double* gv, double* gdx,
                                         double* gdy) {
  constexpr int NW = DEG + 1;
#pragma unroll
  for (int f = 0; f < NF; ++f) gv[f] = gdx[f] = gdy[f] = 0.0;
#pragma unroll
  for (int b = 0; b < NW; ++b) {
    const size_t row = wrap ? (size_t)wrapi(sy + b, g.ny) * g.nx : (size_t)(sy + b) * pitch;
    double aw[NF], ad[NF];
#pragma unroll
    for (int f = 0; f < NF; ++f) aw[f] = ad[f] = 0.0;
#pragma unroll
    for (int a = 0; a < NW; ++a) {
      const size_t m = row + (wrap ? wrapi(sx + a, g.nx) : sx + a);
#pragma unroll
      for (int f = 0; f < NF; ++f) {
        const double v = F[f * stride + m];
        aw[f] += wx[a] * v;
        ad[f] += dwx[a] * v;
      }
    }
#pragma unroll
    for (int f = 0; f < NF; ++f) {
      gv[f] += wy[b] * aw[f];
      gdx[f] += wy[b] * ad[f];
      gdy[f] += dwy[b] * aw[f];
    }
  }
}

// ---------------------------------------------------------------------------
// push + gather adjoint.  Particle arrays hold x^{n+1} (recomputed), P^n, v^n
// and v^{n-1}; F64 holds the mesh fields of level n+1.
template <int DEG>
__global__ void __launch_bounds__(256) k_adj_push(const InstDesc* __restrict__ D, StepArgs sa, double* lam_,
                                                  int64_t ls) {
  using S = Spline<double, DEG>;
  const InstDesc& d = D[0];
  const int64_t n = d.n;
  const int64_t i0 = (int64_t)blockIdx.x * 256, i = i0 + threadIdx.x;
  if (i >= n) return;
  const GridP g = d.g;
  const PhysP ph = d.ph;
  const GParts<double> p = global_parts(make_parts<double>(d, sa.cur, sa.vflip));
  const LamRef lam{gp(lam_) + i0, ls, threadIdx.x};
  const size_t plane = (size_t)g.nx * g.ny;
  const gptr<const double> F = gp((const double*)d.F64);
  const double xi = p.x[i] * g.inv_dx, eta = p.y[i] * g.inv_dy;
  const bool inside = in_box(xi, eta, g);
  int sx = 0, sy = 0;
  double wx[S::NW], dwx[S::NW], wy[S::NW], dwy[S::NW];
  double gv[11], gdx[11], gdy[11];
#pragma unroll
  for (int f = 0; f < 11; ++f) gv[f] = gdx[f] = gdy[f] = 0.0;
  if (inside) {
    S::eval_d(xi, sx, wx, dwx);
    S::eval_d(eta, sy, wy, dwy);
    gather_d<DEG, 11>(F, plane, wx, dwx, wy, dwy, sx, sy, g, 0, true, gv, gdx, gdy);
  }
  double lg[11];
  adj_push_one(gv, p.P[0][i], p.P[1][i], p.P[2][i], p.v[0][i], p.v[1][i], p.v[2][i], p.w[0][i], p.w[1][i],
               p.w[2][i], ph, lam, lg);
  if (!inside) return;
  double lxg = 0.0, lyg = 0.0;
#pragma unroll
  for (int f = 0; f < 11; ++f) {
    lxg += lg[f] * gdx[f];
    lyg += lg[f] * gdy[f];
  }
  lam(0) += lxg * g.inv_dx;  // lambda of x^{n+1}, deposit part still to come
  lam(1) += lyg * g.inv_dy;
  const gptr<double> LF = gp(d.LF);
#pragma unroll
  for (int b = 0; b < S::NW; ++b) {
    const size_t row = (size_t)wrapi(sy + b, g.ny) * g.nx;
#pragma unroll
    for (int a = 0; a < S::NW; ++a) {
      const size_t m = row + wrapi(sx + a, g.nx);
      const double w = wx[a] * wy[b];
#pragma unroll
      for (int f = 0; f < 11; ++f) gadd(LF + f * plane + m, lg[f] * w);
    }
  }
}

// ---------------------------------------------------------------------------
// The same two particle passes over the cell-sorted chunks of the forward
// (one workgroup per chunk, the tile's W x W window in LDS): the push adjoint
// gathers the mesh fields from the window and scatters lambda_g into an LDS
// window of the field adjoints (flushed to LF once per chunk); the deposit
// adjoint gathers lambda_J from a window.  A particle whose stencil leaves the
// window uses the global arrays, as in the forward passes.
struct AdjWin {
  int W, WP, ox, oy, wi, wj0, wjs, gxw;
};

__device__ __forceinline__ AdjWin adj_window(const InstDesc& d, const int4& it) {
  const TileP tp = d.tp;
  AdjWin a;
  a.W = tp.win;
  a.WP = tp.win_pad;
  const int tiy = it.x >> tp.log_ntx, tix = it.x - (tiy << tp.log_ntx);
  a.ox = tix * tp.ts - tp.slack - 1;
  a.oy = tiy * tp.ts - tp.slack - 1;
  a.wi = threadIdx.x & (tp.row_lanes - 1);
  a.wj0 = threadIdx.x >> tp.log_row_lanes;
  a.wjs = blockDim.x >> tp.log_row_lanes;
  a.gxw = (a.ox + a.wi) & (d.g.nx - 1);
  return a;
}

// copy nf planes of the mesh array src[f][ny][nx] into the window dst[f][WP]
__device__ __forceinline__ void adj_load_window(double* __restrict__ dst, gptr<const double> src, int nf,
                                                const AdjWin& a, const GridP& g) {
  const size_t plane = (size_t)g.nx * g.ny;
  if (a.wi < a.W)
    for (int j = a.wj0; j < a.W; j += a.wjs) {
      const size_t go = (size_t)((a.oy + j) & (g.ny - 1)) * g.nx + a.gxw;
      const int node = j * a.W + a.wi;
      for (int f = 0; f < nf; ++f) dst[f * a.WP + node] = src[f * plane + go];
    }
}

// 512 threads: the two LDS windows (about 112 KB at 16-cell tiles) admit one
// workgroup per CU, so the workgroup itself brings the waves that hide latency
// (at most 256 VGPRs each: two waves per SIMD)
constexpr int kAdjPushThreads = 512;

// the work item of this workgroup, its fields wave-uniform (scalar
// registers: the particle arrays' bases offset by its first particle stay
// scalar)
__device__ __forceinline__ int4 adj_item(const InstDesc& d) {
  const int4 w = d.tb.work[blockIdx.x];
  return make_int4(__builtin_amdgcn_readfirstlane(w.x), __builtin_amdgcn_readfirstlane(w.y),
                   __builtin_amdgcn_readfirstlane(w.z), 0);
}

template <int DEG, int TS, int SL>
__global__ void __launch_bounds__(kAdjPushThreads) k_adj_push_t(const InstDesc* __restrict__ D, StepArgs sa,
                                                                double* lam_, int64_t ls) {
  using S = Spline<double, DEG>;
  constexpr int NW = S::NW;
  constexpr bool FIXED = TS > 0;  // compiled window geometry: immediate LDS offsets
  using G = Geo<(FIXED ? TS : 1), (FIXED ? SL : 0)>;
  const InstDesc& d = D[0];
  if ((int)blockIdx.x >= *d.tb.nwork) return;
  const int4 it = adj_item(d);
  const int first = it.y, count = it.z;
  const GridP g = d.g;
  const PhysP ph = d.ph;
  const GParts<double> pall = global_parts(make_parts<double>(d, sa.cur, sa.vflip));
  const gptr<const double> F = gp((const double*)d.F64);
  const gptr<double> LF = gp(d.LF);
  const size_t plane = (size_t)g.nx * g.ny;
  extern __shared__ double2 sm[];
  double* fw = reinterpret_cast<double*>(sm);  // [11][WP] mesh fields of level n+1
  const int lane = threadIdx.x & 63;
  const AdjWin a = adj_window(d, it);
  const int W = FIXED ? G::W : a.W, WP = FIXED ? G::WP : a.WP;
  double* lw = fw + 11 * WP;  // [11][WP] their adjoints
  adj_load_window(fw, F, 11, a, g);
  for (int t = threadIdx.x; t < 11 * WP; t += blockDim.x) lw[t] = 0.0;
  __syncthreads();
  const GParts<double> p = parts_from(pall, first);
  const gptr<double> lamb = gp(lam_) + first;
  for (int k0 = threadIdx.x; k0 < count; k0 += blockDim.x) {
    const uint32_t k = opaque_index(k0);
    const LamRef lam{lamb, ls, k};
    const double xi = elt(p.x, k) * g.inv_dx, eta = elt(p.y, k) * g.inv_dy;
    const bool inside = in_box(xi, eta, g);
    int sx = 0, sy = 0, lx = 0, ly = 0;
    bool inw = false;
    double wx[NW], dwx[NW], wy[NW], dwy[NW];
    double gv[11], gdx[11], gdy[11];
#pragma unroll
    for (int f = 0; f < 11; ++f) gv[f] = gdx[f] = gdy[f] = 0.0;
    if (inside) {
      S::eval_d(xi, sx, wx, dwx);
      S::eval_d(eta, sy, wy, dwy);
      lx = (sx - a.ox) & (g.nx - 1);
      ly = (sy - a.oy) & (g.ny - 1);
      inw = lx + DEG < W && ly + DEG < W;
      if (inw)
        gather_d<DEG, 11>(fw + ly * W + lx, WP, wx, dwx, wy, dwy, 0, 0, g, W, false, gv, gdx, gdy);
      else
        gather_d<DEG, 11>(F, plane, wx, dwx, wy, dwy, sx, sy, g, 0, true, gv, gdx, gdy);
    }
    double lg[11];
    adj_push_one(gv, elt(p.P[0], k), elt(p.P[1], k), elt(p.P[2], k), elt(p.v[0], k), elt(p.v[1], k),
                 elt(p.v[2], k), elt(p.w[0], k), elt(p.w[1], k), elt(p.w[2], k), ph, lam, lg);
    double lxg = 0.0, lyg = 0.0;
#pragma unroll
    for (int f = 0; f < 11; ++f) {
      lxg += lg[f] * gdx[f];
      lyg += lg[f] * gdy[f];
    }
    lam(0) += lxg * g.inv_dx;  // lambda of x^{n+1}, deposit part still to come
    lam(1) += lyg * g.inv_dy;
    // the scatter visits its stencil in the residue-class order of the
    // forward deposit: at step (a, b) lane l adds to the node whose absolute
    // indices are congruent to (a + l, b + l / NW) modulo NW, so at most
    // 64 / NW^2 lanes meet on one window address, whatever cells the wave's
    // particles are in
    const int ra = ((lane - sx) % NW + NW) % NW, rb = ((lane / NW - sy) % NW + NW) % NW;
    double wxr[NW], wyr[NW];
    int coff[NW], roff[NW];
#pragma unroll
    for (int t = 0; t < NW; ++t) {
      int ia = t + ra, ib = t + rb;
      ia = ia >= NW ? ia - NW : ia;
      ib = ib >= NW ? ib - NW : ib;
      wxr[t] = wx[t];
      wyr[t] = wy[t];
      coff[t] = ia;
      roff[t] = ib * W;
    }
    rotate_lanes<NW>(wxr, ra);
    rotate_lanes<NW>(wyr, rb);
    if (inw) {
      double* nd0 = lw + ly * W + lx;
#pragma unroll
      for (int tb = 0; tb < NW; ++tb) {
#pragma unroll
        for (int ta = 0; ta < NW; ++ta) {
          const double w = wxr[ta] * wyr[tb];
          double* nd = nd0 + roff[tb] + coff[ta];
#pragma unroll
          for (int f = 0; f < 11; ++f) atomicAdd(nd + f * WP, lg[f] * w);
        }
      }
    } else if (inside) {
#pragma unroll
      for (int b = 0; b < NW; ++b) {
        const size_t row = (size_t)wrapi(sy + b, g.ny) * g.nx;
#pragma unroll
        for (int aa = 0; aa < NW; ++aa) {
          const size_t m = row + wrapi(sx + aa, g.nx);
          const double w = wx[aa] * wy[b];
#pragma unroll
          for (int f = 0; f < 11; ++f) gadd(LF + f * plane + m, lg[f] * w);
        }
      }
    }
  }
  __syncthreads();
  if (a.wi < W)
    for (int j = a.wj0; j < W; j += a.wjs) {
      const size_t go = (size_t)((a.oy + j) & (g.ny - 1)) * g.nx + a.gxw;
      const int node = j * W + a.wi;
      for (int f = 0; f < 11; ++f) {
        const double v = lw[f * WP + node];
        if (v != 0.0) gadd(LF + f * plane + go, v);
      }
    }
}

template <int DEG, int TS, int SL>
__global__ void __launch_bounds__(256) k_adj_deposit_t(const InstDesc* __restrict__ D, StepArgs sa,
                                                       double* lam_, int64_t ls) {
  using S = Spline<double, DEG>;
  constexpr int NW = S::NW;
  constexpr bool FIXED = TS > 0;  // compiled window geometry: immediate LDS offsets
  using G = Geo<(FIXED ? TS : 1), (FIXED ? SL : 0)>;
  const InstDesc& d = D[0];
  if ((int)blockIdx.x >= *d.tb.nwork) return;
  const int4 it = adj_item(d);
  const int first = it.y, count = it.z;
  const GridP g = d.g;
  const PhysP ph = d.ph;
  const GParts<double> pall = global_parts(make_parts<double>(d, sa.cur, sa.vflip));
  const gptr<const double> LJ = gp((const double*)d.LJ);
  const size_t plane = (size_t)g.nx * g.ny;
  extern __shared__ double2 sm[];
  double* jw = reinterpret_cast<double*>(sm);  // [3][WP] lambda_J
  const double s = ph.q * g.inv_area;
  const AdjWin a = adj_window(d, it);
  const int W = FIXED ? G::W : a.W, WP = FIXED ? G::WP : a.WP;
  adj_load_window(jw, LJ, 3, a, g);
  __syncthreads();
  const GParts<double> p = parts_from(pall, first);
  const gptr<double> lamb = gp(lam_) + first;
  for (int k0 = threadIdx.x; k0 < count; k0 += blockDim.x) {
    const uint32_t k = opaque_index(k0);
    const LamRef lam{lamb, ls, k};
    const double xi = elt(p.x, k) * g.inv_dx, eta = elt(p.y, k) * g.inv_dy;
    double av[3] = {0, 0, 0}, bx[3] = {0, 0, 0}, by[3] = {0, 0, 0};
    if (in_box(xi, eta, g)) {
      int sx, sy;
      double wx[NW], dwx[NW], wy[NW], dwy[NW];
      S::eval_d(xi, sx, wx, dwx);
      S::eval_d(eta, sy, wy, dwy);
      const int lx = (sx - a.ox) & (g.nx - 1), ly = (sy - a.oy) & (g.ny - 1);
      if (lx + DEG < W && ly + DEG < W)
        gather_d<DEG, 3>(jw + ly * W + lx, WP, wx, dwx, wy, dwy, 0, 0, g, W, false, av, bx, by);
      else
        gather_d<DEG, 3>(LJ, plane, wx, dwx, wy, dwy, sx, sy, g, 0, true, av, bx, by);
    }
    const double v0 = elt(p.v[0], k), v1 = elt(p.v[1], k), v2 = elt(p.v[2], k);
    const double lx_ = lam(0) + s * (v0 * bx[0] + v1 * bx[1] + v2 * bx[2]) * g.inv_dx;
    const double ly_ = lam(1) + s * (v0 * by[0] + v1 * by[1] + v2 * by[2]) * g.inv_dy;
    lam(0) = lx_;
    lam(1) = ly_;
    lam(5) += s * av[0] + ph.dt * lx_;
    lam(6) += s * av[1] + ph.dt * ly_;
    lam(7) += s * av[2];
  }
}

// ---------------------------------------------------------------------------
// columns of the field-solve adjoint: one block per kx.
// In:  LS[f][kx][y]   x-transforms of the 11 mesh-field adjoints
//      lamH           adjoint of the history after the update (external
//                     layout [field][ky][kx]; BDF-k order: rho (k levels),
//                     phi (2k), A (2k levels x 3 components))
// Out: lamH           adjoint of the history before the update (in place)
//      LS[c][kx][y]   c < 3: y-inverse transforms of lambda_J^ / w
// Mesh field f is irfft2(sigma_f X_src(f)) with X = phi or A_l and sigma one
// of 1, i kx, i ky (the forward column and row kernels); its adjoint adds
// conj(sigma_f) (w / N) rfft2(lambda_F_f) to lambda_X.
__constant__ int kAdjSrc[11] = {0, 0, 1, 2, 3, 1, 2, 3, 1, 2, 3};  // 0 phi, 1..3 A_l
__constant__ int kAdjSym[11] = {1, 2, 0, 0, 0, 1, 1, 1, 2, 2, 2};  // 0: 1, 1: i kx, 2: i ky

template <int K>  // the BDF order (static history indices)
__global__ void __launch_bounds__(256) k_adj_columns(const InstDesc* __restrict__ D, double2* __restrict__ lamH) {
  // LDS: acc [0, 4N) = lambda of phi^{n+1}, A_l^{n+1} from the mesh fields;
  // work buffers from 4N: 2 x NB*N (forward batches), 2 x 3N (inverse); then
  // the N twiddles (ny <= 512)
  extern __shared__ double2 sm[];
  const InstDesc& d = D[0];
  const GridP g = d.g;
  const SchemeCoef sc = d.sc;
  const int kx = blockIdx.x;
  const int N = g.ny, NB = d.nb_col, nxh = g.nxh;
  double2* __restrict__ LS = d.LS;
  double2* acc = sm;
  double2* wk = sm + 4 * N;
  // twiddles staged in LDS where they fit (ny <= 512), else read from global
  const double2* tws = d.twy;
  if (N <= 512) {
    double2* t_lds = wk + max(6, 2 * NB) * N;
    for (int t = threadIdx.x; t < N; t += blockDim.x) t_lds[t] = d.twy[t];
    tws = t_lds;
  }
  const double wgt = (kx == 0 || 2 * kx == g.nx) ? 1.0 : 2.0;
  const double norm = wgt / ((double)g.nx * g.ny);
  const double kxs = kx_sym(kx, g);
  for (int t = threadIdx.x; t < 4 * N; t += blockDim.x) acc[t] = make_double2(0.0, 0.0);
  for (int f0 = 0; f0 < 11; f0 += NB) {
    const int nb = min(NB, 11 - f0);
    for (int t = threadIdx.x; t < nb * N; t += blockDim.x) {
      const int qf = t / N, y = t - qf * N;
      wk[t] = LS[((size_t)(f0 + qf) * nxh + kx) * N + y];
    }
    __syncthreads();
    const double2* res = fft_lds<false>(wk, wk + nb * N, N, nb, tws);
    // each thread owns its ky entries of acc: the field loop is serial
    for (int ky = threadIdx.x; ky < N; ky += blockDim.x) {
      const double kys = ky_sym(ky, g);
      for (int qf = 0; qf < nb; ++qf) {
        const int f = f0 + qf;
        double2 z = cscale(res[qf * N + ky], norm);
        const int sy = kAdjSym[f];
        if (sy == 1) z = mul_mi(cscale(z, kxs));       // conj(i kx) = -i kx
        else if (sy == 2) z = mul_mi(cscale(z, kys));  // conj(i ky) = -i ky
        double2& a = acc[kAdjSrc[f] * N + ky];
        a = cadd(a, z);
      }
    }
    __syncthreads();
  }
  // transposed per-mode BDF-k update.  Forward (per mode, Lh = 1 + kappa/alpha^2):
  //   rho' = -(sum_{j=1..k} a_j R_{j-1} + dt i k.J^) / a_0
  //   phi' = (rho' / (eps0 alpha^2) - sum_{i=1..2k} Cn_i Phi_{i-1}) / Lh
  //   A'_l = (mu0 J^_l / alpha^2 - sum_{i=1..2k} Cn_i A_{i-1,l}) / Lh
  //   history shift: R <- (rho', R_0 .. R_{k-2}), Phi and A likewise
  constexpr int k = K;
  const size_t fstride = (size_t)N * nxh;
  for (int ky = threadIdx.x; ky < N; ky += blockDim.x) {
    const double kys = ky_sym(ky, g);
    const double Lh = 1.0 + (kxs * kxs + kys * kys) * sc.inv_alpha2;
    double2* h = lamH + (size_t)ky * nxh + kx;
    auto R = [&](int j) -> double2& { return h[(size_t)j * fstride]; };
    auto Ph = [&](int j) -> double2& { return h[(size_t)(k + j) * fstride]; };
    auto Al = [&](int j, int l) -> double2& { return h[(size_t)(3 * k + 3 * j + l) * fstride]; };
    const double2 lphi = cadd(Ph(0), acc[ky]);
    double2 lA[3];
    for (int l = 0; l < 3; ++l) lA[l] = cadd(Al(0, l), acc[(1 + l) * N + ky]);
    const double2 lrho = cadd(R(0), cscale(lphi, sc.inv_alpha2 / (sc.eps0 * Lh)));
    // shifts (ascending: slot j is read before it is overwritten)
#pragma unroll
    for (int i = 1; i <= 2 * k; ++i) {
      const double2 up = i < 2 * k ? Ph(i) : make_double2(0.0, 0.0);
      Ph(i - 1) = csub(up, cscale(lphi, sc.Cn[i] / Lh));
    }
    for (int l = 0; l < 3; ++l)
#pragma unroll
      for (int i = 1; i <= 2 * k; ++i) {
        const double2 up = i < 2 * k ? Al(i, l) : make_double2(0.0, 0.0);
        Al(i - 1, l) = csub(up, cscale(lA[l], sc.Cn[i] / Lh));
      }
#pragma unroll
    for (int j = 1; j <= k; ++j) {
      const double2 up = j < k ? R(j) : make_double2(0.0, 0.0);
      R(j - 1) = csub(up, cscale(lrho, sc.a[j] / sc.a[0]));
    }
    // lambda_J^_l = mu0/(alpha^2 Lh) lambda_A'_l + conj(-dt i k_l / a_0) lambda_rho'
    const double cA = sc.mu0 * sc.inv_alpha2 / Lh;
    const double cr = sc.dt / sc.a[0];
    const double2 lJx = cadd(cscale(lA[0], cA), mul_i(cscale(lrho, cr * kxs)));
    const double2 lJy = cadd(cscale(lA[1], cA), mul_i(cscale(lrho, cr * kys)));
    const double2 lJz = cscale(lA[2], cA);
    // lambda_J = N irfft2(lambda_J^ / w): the y-inverse here, the rows next
    wk[ky] = cscale(lJx, 1.0 / wgt);
    wk[N + ky] = cscale(lJy, 1.0 / wgt);
    wk[2 * N + ky] = cscale(lJz, 1.0 / wgt);
  }
  __syncthreads();
  const double2* res = fft_lds<true>(wk, wk + 3 * N, N, 3, tws);
  for (int t = threadIdx.x; t < 3 * N; t += blockDim.x) {
    const int c = t / N, y = t - c * N;
    LS[((size_t)c * nxh + kx) * N + y] = res[t];
  }
}

// ---------------------------------------------------------------------------
// deposit adjoint + position update adjoint.  Particle arrays hold x^{n+1}
// and v^n; LJ holds lambda_J.
template <int DEG>
__global__ void __launch_bounds__(256) k_adj_deposit(const InstDesc* __restrict__ D, StepArgs sa, double* lam_,
                                                     int64_t ls) {
  using S = Spline<double, DEG>;
  const InstDesc& d = D[0];
  const int64_t n = d.n;
  const int64_t i0 = (int64_t)blockIdx.x * 256, i = i0 + threadIdx.x;
  if (i >= n) return;
  const GridP g = d.g;
  const PhysP ph = d.ph;
  const GParts<double> p = global_parts(make_parts<double>(d, sa.cur, sa.vflip));
  const LamRef lam{gp(lam_) + i0, ls, threadIdx.x};
  const size_t plane = (size_t)g.nx * g.ny;
  const gptr<const double> LJ = gp((const double*)d.LJ);
  const double xi = p.x[i] * g.inv_dx, eta = p.y[i] * g.inv_dy;
  double av[3] = {0, 0, 0}, bx[3] = {0, 0, 0}, by[3] = {0, 0, 0};
  if (in_box(xi, eta, g)) {
    int sx, sy;
    double wx[S::NW], dwx[S::NW], wy[S::NW], dwy[S::NW];
    S::eval_d(xi, sx, wx, dwx);
    S::eval_d(eta, sy, wy, dwy);
#pragma unroll
    for (int b = 0; b < S::NW; ++b) {
      const size_t row = (size_t)wrapi(sy + b, g.ny) * g.nx;
      double aw[3] = {0, 0, 0}, ad[3] = {0, 0, 0};
#pragma unroll
      for (int a = 0; a < S::NW; ++a) {
        const size_t m = row + wrapi(sx + a, g.nx);
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          const double v = LJ[c * plane + m];
          aw[c] += wx[a] * v;
          ad[c] += dwx[a] * v;
        }
      }
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        av[c] += wy[b] * aw[c];
        bx[c] += wy[b] * ad[c];
        by[c] += dwy[b] * aw[c];
      }
    }
  }
  // J = sum q v^n S(x' - X) / (dx dy)
  const double s = ph.q * g.inv_area;
  const double v0 = p.v[0][i], v1 = p.v[1][i], v2 = p.v[2][i];
  const double lx = lam(0) + s * (v0 * bx[0] + v1 * bx[1] + v2 * bx[2]) * g.inv_dx;
  const double ly = lam(1) + s * (v0 * by[0] + v1 * by[1] + v2 * by[2]) * g.inv_dy;
  // x' = wrap(x + v^n dt): unit derivative in x, dt in v
  lam(0) = lx;
  lam(1) = ly;
  lam(5) += s * av[0] + ph.dt * lx;
  lam(6) += s * av[1] + ph.dt * ly;
  lam(7) += s * av[2];
}

// ---------------------------------------------------------------------------
// adjoint of the field energy of the newest level (BDF-k time derivative):
//   W = (dx dy / 2N) sum_modes w (eps0 |E^|^2 + |B^|^2 / mu0),
//   E^ = -i k phi^n - (1/dt) sum_j a_j A^{n-j},  B^ = i k x A^n,
// the Parseval form of the mesh sum of (eps0 |E|^2 + |B|^2/mu0) dx dy / 2.
// Writes scale * dW/dH for every external history field.
__global__ void k_adj_seed_energy(const double2* __restrict__ H, GridP g, SchemeCoef sc, HistSlots hs, double scale,
                                  double2* __restrict__ lamH, int nf) {
  const size_t plane = (size_t)g.nxh * g.ny;
  const int k = sc.k;
  for (size_t t = blockIdx.x * (size_t)blockDim.x + threadIdx.x; t < plane; t += (size_t)gridDim.x * blockDim.x) {
    const int ky = (int)(t / g.nxh), kx = (int)(t - (size_t)ky * g.nxh);
    const size_t m = (size_t)kx * g.ny + ky;  // internal [kx][ky]
    const double kxs = kx_sym(kx, g), kys = ky_sym(ky, g);
    const double wgt = (kx == 0 || 2 * kx == g.nx) ? 1.0 : 2.0;
    const double s = scale * wgt * g.dx * g.dy / ((double)g.nx * g.ny);
    auto at = [&](int slot) { return H[(size_t)slot * plane + m]; };
    const double2 phi = at(hs.phi[0]);
    double2 dA[3] = {{0, 0}, {0, 0}, {0, 0}};
    for (int j = 0; j <= k; ++j)
      for (int l = 0; l < 3; ++l) dA[l] = cadd(dA[l], cscale(at(hs.A[j] + l), sc.a[j] / sc.dt));
    double2 A0[3];
    for (int l = 0; l < 3; ++l) A0[l] = at(hs.A[0] + l);
    const double2 Ex = csub(mul_i(cscale(phi, -kxs)), dA[0]);
    const double2 Ey = csub(mul_i(cscale(phi, -kys)), dA[1]);
    const double2 Ez = cscale(dA[2], -1.0);
    const double2 Bx = mul_i(cscale(A0[2], kys)), By = mul_i(cscale(A0[2], -kxs));
    const double2 Bz = mul_i(make_double2(kxs * A0[1].x - kys * A0[0].x, kxs * A0[1].y - kys * A0[0].y));
    const double2 lE[3] = {cscale(Ex, s * sc.eps0), cscale(Ey, s * sc.eps0), cscale(Ez, s * sc.eps0)};
    const double2 lBx = cscale(Bx, s / sc.mu0), lBy = cscale(By, s / sc.mu0), lBz = cscale(Bz, s / sc.mu0);
    for (int f = 0; f < nf; ++f) lamH[(size_t)f * plane + t] = make_double2(0.0, 0.0);
    // phi^n: conj(-i k) = i k
    lamH[(size_t)k * plane + t] = mul_i(make_double2(kxs * lE[0].x + kys * lE[1].x, kxs * lE[0].y + kys * lE[1].y));
    for (int j = 0; j <= k; ++j)
      for (int l = 0; l < 3; ++l) {
        double2 v = cscale(lE[l], -sc.a[j] / sc.dt);
        if (j == 0) {  // curl A^n
          if (l == 0) v = cadd(v, mul_i(cscale(lBz, kys)));
          if (l == 1) v = cadd(v, mul_i(cscale(lBz, -kxs)));
          if (l == 2) v = cadd(v, mul_i(make_double2(kxs * lBy.x - kys * lBx.x, kxs * lBy.y - kys * lBx.y)));
        }
        lamH[(size_t)(3 * k + 3 * j + l) * plane + t] = v;
      }
  }
}

// adjoint of the cold start v^0 = v^{-1} = c^2 P / sqrt(c^2 |P|^2 + (m c^2)^2):
// lambda_P += J^T (lambda_{v^0} + lambda_{v^{-1}}), velocity adjoints cleared
__global__ void k_adj_initial(int64_t n, const double* __restrict__ P, PhysP ph, double* __restrict__ lam) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double c2 = ph.c * ph.c, mc2 = ph.m * c2;
  const double ux = P[i], uy = P[n + i], uz = P[2 * n + i];
  const double ss = sqrt(c2 * (ux * ux + uy * uy + uz * uz) + mc2 * mc2);
  const double lvx = lam[5 * n + i] + lam[8 * n + i];
  const double lvy = lam[6 * n + i] + lam[9 * n + i];
  const double lvz = lam[7 * n + i] + lam[10 * n + i];
  const double ud = (ux * lvx + uy * lvy + uz * lvz) * c2 / (ss * ss);
  const double k1 = c2 / ss;
  lam[2 * n + i] += k1 * (lvx - ud * ux);
  lam[3 * n + i] += k1 * (lvy - ud * uy);
  lam[4 * n + i] += k1 * (lvz - ud * uz);
  for (int c = 5; c < 11; ++c) lam[c * n + i] = 0.0;
}

// ---------------------------------------------------------------------------
// The held particle adjoint.  k_lam_set: from original order (lam[11][n]),
// slot i holding particle i; null: zero, in the slot order of the set the
// passes run on (ids), so that no permutation follows.  k_lam_get: back to
// original order.
__global__ void k_lam_set(int64_t n, const double* __restrict__ src, double* __restrict__ LAM, int64_t ls,
                          int32_t* __restrict__ LIDS, const int32_t* __restrict__ ids) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= n) return;
  for (int f = 0; f < 11; ++f) LAM[f * ls + i] = src ? src[f * n + i] : 0.0;
  LIDS[i] = src ? (int32_t)i : ids[i];
}

__global__ void k_lam_get(int64_t n, const double* __restrict__ LAM, int64_t ls, const int32_t* __restrict__ LIDS,
                          double* __restrict__ dst) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int64_t o = LIDS[i];
  for (int f = 0; f < 11; ++f) dst[f * n + o] = LAM[f * ls + i];
}

// Following the particle set's order: flag = (LIDS differs from ids anywhere);
// then, only if set, LINV = the slot of each particle in LAM, LAM2 = LAM in
// the order of ids, and LAM, LIDS = LAM2, ids.  The host never reads the flag,
// so a step without a sort costs one pass over the two index arrays.
__global__ void k_lam_flag_clear(int32_t* flag) {
  if (threadIdx.x == 0) *flag = 0;
}

__global__ void k_lam_check(int64_t n, const int32_t* __restrict__ LIDS, const int32_t* __restrict__ ids,
                            int32_t* flag) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  const bool diff = i < n && LIDS[i] != ids[i];
  if (__any(diff) && (threadIdx.x & 63) == 0) *flag = 1;
}

__global__ void k_lam_inverse(int64_t n, const int32_t* __restrict__ LIDS, int32_t* __restrict__ LINV,
                              const int32_t* flag) {
  if (!*flag) return;
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < n) LINV[LIDS[i]] = (int32_t)i;
}

__global__ void k_lam_permute(int64_t n, const double* __restrict__ LAM, double* __restrict__ LAM2, int64_t ls,
                              const int32_t* __restrict__ ids, const int32_t* __restrict__ LINV,
                              const int32_t* flag) {
  if (!*flag) return;
  const int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (j >= n) return;
  const int64_t src = LINV[ids[j]];
  for (int f = 0; f < 11; ++f) LAM2[f * ls + j] = LAM[f * ls + src];
}

__global__ void k_lam_commit(int64_t n, const double* __restrict__ LAM2, double* __restrict__ LAM, int64_t ls,
                             const int32_t* __restrict__ ids, int32_t* __restrict__ LIDS, const int32_t* flag) {
  if (!*flag) return;
  const int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (j >= n) return;
  for (int f = 0; f < 11; ++f) LAM[f * ls + j] = LAM2[f * ls + j];
  LIDS[j] = ids[j];
}

inline unsigned blocks_for(int64_t n) { return (unsigned)((n + 255) / 256); }

}  // namespace

hipError_t launch_lam_set(int64_t n, const double* src, double* LAM, int64_t ls, int32_t* LIDS, const int32_t* ids,
                          hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_lam_set, dim3(blocks_for(n)), dim3(256), 0, s, n, src, LAM, ls, LIDS, ids);
  return hipGetLastError();
}

hipError_t launch_lam_get(int64_t n, const double* LAM, int64_t ls, const int32_t* LIDS, double* dst, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_lam_get, dim3(blocks_for(n)), dim3(256), 0, s, n, LAM, ls, LIDS, dst);
  return hipGetLastError();
}

hipError_t launch_lam_follow(int64_t n, const int32_t* ids, double* LAM, double* LAM2, int64_t ls, int32_t* LIDS,
                             int32_t* LINV, int32_t* flag, hipStream_t s) {
  if (n == 0) return hipSuccess;
  const dim3 grid(blocks_for(n)), block(256);
  hipLaunchKernelGGL(k_lam_flag_clear, dim3(1), dim3(64), 0, s, flag);
  hipLaunchKernelGGL(k_lam_check, grid, block, 0, s, n, (const int32_t*)LIDS, ids, flag);
  hipLaunchKernelGGL(k_lam_inverse, grid, block, 0, s, n, (const int32_t*)LIDS, LINV, (const int32_t*)flag);
  hipLaunchKernelGGL(k_lam_permute, grid, block, 0, s, n, (const double*)LAM, LAM2, ls, ids, (const int32_t*)LINV,
                     (const int32_t*)flag);
  hipLaunchKernelGGL(k_lam_commit, grid, block, 0, s, n, (const double*)LAM2, LAM, ls, ids, LIDS,
                     (const int32_t*)flag);
  return hipGetLastError();
}

hipError_t launch_adj_push(int degree, const InstDesc* D, int64_t n, StepArgs sa, double* lam, int64_t ls,
                           hipStream_t s) {
  if (n == 0) return hipSuccess;
  switch (degree) {
    case 1: hipLaunchKernelGGL(k_adj_push<1>, dim3(blocks_for(n)), dim3(256), 0, s, D, sa, lam, ls); break;
    case 2: hipLaunchKernelGGL(k_adj_push<2>, dim3(blocks_for(n)), dim3(256), 0, s, D, sa, lam, ls); break;
    default: hipLaunchKernelGGL(k_adj_push<3>, dim3(blocks_for(n)), dim3(256), 0, s, D, sa, lam, ls); break;
  }
  return hipGetLastError();
}

hipError_t launch_adj_deposit(int degree, const InstDesc* D, int64_t n, StepArgs sa, double* lam, int64_t ls,
                              hipStream_t s) {
  if (n == 0) return hipSuccess;
  switch (degree) {
    case 1: hipLaunchKernelGGL(k_adj_deposit<1>, dim3(blocks_for(n)), dim3(256), 0, s, D, sa, lam, ls); break;
    case 2: hipLaunchKernelGGL(k_adj_deposit<2>, dim3(blocks_for(n)), dim3(256), 0, s, D, sa, lam, ls); break;
    default: hipLaunchKernelGGL(k_adj_deposit<3>, dim3(blocks_for(n)), dim3(256), 0, s, D, sa, lam, ls); break;
  }
  return hipGetLastError();
}

size_t adj_tiled_lds_bytes(const TileP& tp, bool push) { return (size_t)(push ? 22 : 3) * tp.win_pad * 8; }

hipError_t launch_adj_tiled(bool push, int degree, int geo, const InstDesc* D, int nblocks, size_t lds, StepArgs sa,
                            double* lam, int64_t ls, hipStream_t s) {
  if (nblocks == 0) return hipSuccess;
  const void* fn = nullptr;
  if (push)
    fn = degree == 1 ? (const void*)k_adj_push_t<1, 0, 0>
         : degree == 2 ? (const void*)k_adj_push_t<2, 0, 0>
         : geo == 1    ? (const void*)k_adj_push_t<3, 16, 3>
         : geo == 2    ? (const void*)k_adj_push_t<3, 8, 3>
                       : (const void*)k_adj_push_t<3, 0, 0>;
  else
    fn = degree == 1 ? (const void*)k_adj_deposit_t<1, 0, 0>
         : degree == 2 ? (const void*)k_adj_deposit_t<2, 0, 0>
         : geo == 1    ? (const void*)k_adj_deposit_t<3, 16, 3>
         : geo == 2    ? (const void*)k_adj_deposit_t<3, 8, 3>
                       : (const void*)k_adj_deposit_t<3, 0, 0>;
  (void)hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (push) {
    const dim3 grid(nblocks), block(kAdjPushThreads);
    if (degree == 1)
      hipLaunchKernelGGL((k_adj_push_t<1, 0, 0>), grid, block, lds, s, D, sa, lam, ls);
    else if (degree == 2)
      hipLaunchKernelGGL((k_adj_push_t<2, 0, 0>), grid, block, lds, s, D, sa, lam, ls);
    else if (geo == 1)
      hipLaunchKernelGGL((k_adj_push_t<3, 16, 3>), grid, block, lds, s, D, sa, lam, ls);
    else if (geo == 2)
      hipLaunchKernelGGL((k_adj_push_t<3, 8, 3>), grid, block, lds, s, D, sa, lam, ls);
    else
      hipLaunchKernelGGL((k_adj_push_t<3, 0, 0>), grid, block, lds, s, D, sa, lam, ls);
  } else {
    const dim3 grid(nblocks), block(256);
    if (degree == 1)
      hipLaunchKernelGGL((k_adj_deposit_t<1, 0, 0>), grid, block, lds, s, D, sa, lam, ls);
    else if (degree == 2)
      hipLaunchKernelGGL((k_adj_deposit_t<2, 0, 0>), grid, block, lds, s, D, sa, lam, ls);
    else if (geo == 1)
      hipLaunchKernelGGL((k_adj_deposit_t<3, 16, 3>), grid, block, lds, s, D, sa, lam, ls);
    else if (geo == 2)
      hipLaunchKernelGGL((k_adj_deposit_t<3, 8, 3>), grid, block, lds, s, D, sa, lam, ls);
    else
      hipLaunchKernelGGL((k_adj_deposit_t<3, 0, 0>), grid, block, lds, s, D, sa, lam, ls);
  }
  return hipGetLastError();
}

template <int K>
static hipError_t launch_adj_columns_t(const InstDesc* D, int nxh, size_t lds, double* lam_hist, hipStream_t s) {
  (void)hipFuncSetAttribute((const void*)k_adj_columns<K>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  hipLaunchKernelGGL(k_adj_columns<K>, dim3(nxh), dim3(256), lds, s, D, (double2*)lam_hist);
  return hipGetLastError();
}

hipError_t launch_adj_columns(int bdf_order, const InstDesc* D, int nxh, size_t lds, double* lam_hist, hipStream_t s) {
  switch (bdf_order) {
    case 1: return launch_adj_columns_t<1>(D, nxh, lds, lam_hist, s);
    case 2: return launch_adj_columns_t<2>(D, nxh, lds, lam_hist, s);
    case 3: return launch_adj_columns_t<3>(D, nxh, lds, lam_hist, s);
    case 4: return launch_adj_columns_t<4>(D, nxh, lds, lam_hist, s);
    case 5: return launch_adj_columns_t<5>(D, nxh, lds, lam_hist, s);
    default: return launch_adj_columns_t<6>(D, nxh, lds, lam_hist, s);
  }
}

hipError_t launch_adj_seed_energy(const double2* H, GridP g, SchemeCoef sc, HistSlots hs, double scale,
                                  double* lam_hist, int nf, hipStream_t s) {
  const size_t plane = (size_t)g.nxh * g.ny;
  const int blocks = (int)std::min<size_t>((plane + 255) / 256, 2048);
  hipLaunchKernelGGL(k_adj_seed_energy, dim3(blocks), dim3(256), 0, s, H, g, sc, hs, scale, (double2*)lam_hist, nf);
  return hipGetLastError();
}

hipError_t launch_adj_initial(int64_t n, const double* P, PhysP ph, double* lam, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_adj_initial, dim3(blocks_for(n)), dim3(256), 0, s, n, P, ph, lam);
  return hipGetLastError();
}

}  // namespace pic
