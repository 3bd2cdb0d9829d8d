// Tile-sorted particle passes with LDS-privatised gather and deposition.
//
// The grid's cells are split into tiles of TS x TS cells.  Every few steps the
// particles are counting-sorted by the tile of their position (k_tile_count,
// k_tile_scan, k_tile_scatter), and the scan cuts each tile's particle range
// into chunks of at most CH particles: one chunk per workgroup.
//
// A workgroup owns a window of W x W mesh nodes around its tile: the tile's
// TS cells, a slack of S cells on each side (particles drift after the sort),
// and the widest stencil reach (one node below, two above the cell).  It
// copies the eleven gathered fields of the window into LDS, node-interleaved,
// gathers from there, accumulates its J contributions in an LDS window, and
// adds that window to the global float64 J with one atomic per non-zero node
// component.  A particle whose stencil leaves the window (it drifted further
// than S cells since the sort) takes the global-memory path for that
// operation, so results never depend on the sort.
//
// The per-particle arithmetic (spline weights, IAEM push, position update) is
// shared with the untiled kernels through particle_math.h.
#include "particle_math.h"

namespace pic {

namespace {

constexpr int kThreads = 256;

// tile of a position (cells floor(xi), clamped into the grid)
__device__ __forceinline__ int tile_of(float xi, float eta, const TileP& tp) {
  int cx = (int)floorf(xi), cy = (int)floorf(eta);
  cx = cx < 0 ? 0 : (cx >= tp.nx ? tp.nx - 1 : cx);
  cy = cy < 0 ? 0 : (cy >= tp.ny ? tp.ny - 1 : cy);
  return (cy >> tp.log_ts) * tp.ntx + (cx >> tp.log_ts);
}

template <typename T>
__device__ __forceinline__ int tile_key(T x, T y, const GridP& g, const TileP& tp) {
  const float xi = (float)(x * T(g.inv_dx)), eta = (float)(y * T(g.inv_dy));
  const bool ok = xi == xi && eta == eta;  // non-finite positions go to tile 0
  return ok ? tile_of(xi, eta, tp) : 0;
}

// Lanes of one wave that share a key: one LDS atomic per distinct key in the
// wave (particles are nearly sorted between sorts, so a wave holds few keys).
// Returns the lane's rank among the wave's lanes with its key, and the value
// the group's atomic returned (the group's base) broadcast to the group.
__device__ __forceinline__ int wave_group_add(int32_t* __restrict__ counters, int key, bool active, int& rank) {
  const int lane = threadIdx.x & 63;
  uint64_t pending = __ballot(active);
  int base = 0;
  rank = 0;
  while (pending) {
    const int leader = __ffsll((unsigned long long)pending) - 1;
    const int k0 = __shfl(key, leader);
    const uint64_t grp = __ballot(active && key == k0);
    int b = 0;
    if (lane == leader) b = atomicAdd(&counters[k0], __popcll(grp));
    b = __shfl(b, leader);
    if (active && key == k0) {
      base = b;
      rank = __popcll(grp & ((1ull << lane) - 1ull));
    }
    pending &= ~grp;
  }
  return base;
}

// Tile histogram of the current positions: each block counts 1024 particles
// of one instance (flattened over instances, BK_COUNT).
template <typename T>
__global__ void __launch_bounds__(kThreads) k_tile_count(const InstDesc* __restrict__ D, int ninst, int set) {
  extern __shared__ int32_t hist[];  // ntiles of this instance
  const int ii = find_inst(D, ninst, BK_COUNT, blockIdx.x);
  const InstDesc& d = D[ii];
  const TileP tp = d.tp;
  const GridP g = d.g;
  const T* __restrict__ px = (const T*)d.set[set][0];
  const T* __restrict__ py = (const T*)d.set[set][1];
  for (int t = threadIdx.x; t < tp.ntiles; t += blockDim.x) hist[t] = 0;
  __syncthreads();
  const int64_t base = (int64_t)(blockIdx.x - d.blk[BK_COUNT]) * 1024;
  for (int k = 0; k < 4; ++k) {  // whole waves stay in the loop
    const int64_t i = base + k * kThreads + threadIdx.x;
    const bool act = i < d.n;
    int t = 0;
    if (act) t = tile_key(px[i], py[i], g, tp);
    int r;
    wave_group_add(hist, t, act, r);
  }
  __syncthreads();
  for (int t = threadIdx.x; t < tp.ntiles; t += blockDim.x)
    if (hist[t]) atomicAdd(&d.tb.count[t], hist[t]);
}

// one block per instance: exclusive scan of the tile counts, cursors, chunk list
__global__ void __launch_bounds__(1024) k_tile_scan(const InstDesc* __restrict__ D, int ninst) {
  __shared__ int32_t s_cnt[1024], s_chk[1024];
  __shared__ int32_t carry_p, carry_c;
  const InstDesc& d = D[blockIdx.x];
  const TileP tp = d.tp;
  int32_t* __restrict__ count = d.tb.count;
  if (threadIdx.x == 0) {
    carry_p = 0;
    carry_c = 0;
  }
  __syncthreads();
  for (int base = 0; base < tp.ntiles; base += 1024) {
    const int t = base + threadIdx.x;
    const int c = t < tp.ntiles ? count[t] : 0;
    const int k = (c + tp.chunk - 1) / tp.chunk;
    s_cnt[threadIdx.x] = c;
    s_chk[threadIdx.x] = k;
    __syncthreads();
    // Hillis-Steele inclusive scans
    for (int off = 1; off < 1024; off <<= 1) {
      const int a = threadIdx.x >= off ? s_cnt[threadIdx.x - off] : 0;
      const int b = threadIdx.x >= off ? s_chk[threadIdx.x - off] : 0;
      __syncthreads();
      s_cnt[threadIdx.x] += a;
      s_chk[threadIdx.x] += b;
      __syncthreads();
    }
    const int p0 = carry_p + s_cnt[threadIdx.x] - c;  // exclusive
    const int k0 = carry_c + s_chk[threadIdx.x] - k;
    if (t < tp.ntiles) {
      d.tb.start[t] = p0;
      d.tb.cursor[t] = p0;
      for (int j = 0; j < k; ++j) {
        const int s = p0 + j * tp.chunk;
        const int e = min(p0 + c, s + tp.chunk);
        d.tb.work[k0 + j] = make_int4(t, s, e - s, 0);
      }
      count[t] = 0;  // ready for the next sort
    }
    __syncthreads();
    if (threadIdx.x == 1023) {
      carry_p += s_cnt[1023];
      carry_c += s_chk[1023];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    d.tb.start[tp.ntiles] = carry_p;
    *d.tb.nwork = carry_c;
  }
}

// scatter set `src` into set `src ^ 1`; one global atomic per (block, tile)
template <typename T>
__global__ void __launch_bounds__(kThreads) k_tile_scatter(const InstDesc* __restrict__ D, int ninst, int src) {
  extern __shared__ int32_t sh[];  // ntiles local counts, then ntiles bases
  const int ii = find_inst(D, ninst, BK_PART, blockIdx.x);
  const InstDesc& d = D[ii];
  const TileP tp = d.tp;
  int32_t* lc = sh;
  int32_t* lb = sh + tp.ntiles;
  const int64_t i = (int64_t)(blockIdx.x - d.blk[BK_PART]) * kThreads + threadIdx.x;
  for (int t = threadIdx.x; t < tp.ntiles; t += blockDim.x) lc[t] = 0;
  __syncthreads();
  const bool act = i < d.n;
  const void* const* S = d.set[src];
  void* const* Dd = d.set[src ^ 1];
  const int k = act ? tile_key(((const T*)S[0])[i], ((const T*)S[1])[i], d.g, tp) : 0;
  int rr;
  const int r = wave_group_add(lc, k, act, rr) + rr;
  __syncthreads();
  for (int t = threadIdx.x; t < tp.ntiles; t += blockDim.x)
    lb[t] = lc[t] ? atomicAdd(&d.tb.cursor[t], lc[t]) : 0;
  __syncthreads();
  if (act) {
    const int64_t o = lb[k] + r;
#pragma unroll
    for (int a = 0; a < 11; ++a) ((T*)Dd[a])[o] = ((const T*)S[a])[i];
    d.ids[src ^ 1][o] = d.ids[src][i];
  }
}

// ---------------------------------------------------------------------------
// the tiled particle pass

enum { MODE_DEPOSIT = 0, MODE_GATHER_PUSH = 1, MODE_FUSED = 2 };

// LDS accumulator of the deposit: float64 for both particle precisions.  On
// gfx950 the LDS float64 add (ds_add_f64) sustains several times the rate of
// the float32 add, and it keeps the per-tile partial sums exact to float64.
template <typename T>
struct Acc {
  using type = double;
};

template <typename T, int DEG, int MODE>
__global__ void __launch_bounds__(kThreads) k_tiled(const InstDesc* __restrict__ D, int ninst, StepArgs sa) {
  constexpr bool GATHER = MODE != MODE_DEPOSIT;
  constexpr bool DEPOSIT = MODE != MODE_GATHER_PUSH;
  using A = typename Acc<T>::type;
  const int ii = find_inst(D, ninst, BK_WORK, blockIdx.x);
  const InstDesc& d = D[ii];
  const int item = blockIdx.x - d.blk[BK_WORK];
  if (item >= *d.tb.nwork) return;
  const int4 it = d.tb.work[item];
  const GridP g = d.g;
  const PhysP ph = d.ph;
  const TileP tp = d.tp;
  const Parts<T> p = make_parts<T>(d, sa.cur, sa.vflip);
  const T* __restrict__ F = GATHER ? (d.F32 ? (const T*)(const void*)d.F32 : (const T*)(const void*)d.F64) : nullptr;
  double* __restrict__ J = d.J;
  const int W = tp.win;
  const int WP = tp.win_pad;  // plane stride of the LDS windows (field f at f*WP)
  const int tiy = it.x >> tp.log_ntx, tix = it.x - (tiy << tp.log_ntx);
  const int ox = tix * tp.ts - tp.slack - 1, oy = tiy * tp.ts - tp.slack - 1;
  extern __shared__ __align__(16) unsigned char smem[];
  T* fw = reinterpret_cast<T*>(smem);
  A* jw = reinterpret_cast<A*>(smem + (GATHER ? (size_t)11 * WP * sizeof(T) : 0));
  const size_t plane = (size_t)g.nx * g.ny;
  // window sweeps without integer division: lanes of a row-group cover x
  // (tp.row_lanes >= W, a power of two), row-groups cover y
  const int rl = tp.row_lanes, lrl = tp.log_row_lanes;
  const int wi = threadIdx.x & (rl - 1), wj0 = threadIdx.x >> lrl, wjs = blockDim.x >> lrl;
  const int gxw = (ox + wi) & (g.nx - 1);
  if (GATHER && wi < W) {
    for (int j = wj0; j < W; j += wjs) {
      const size_t go = (size_t)((oy + j) & (g.ny - 1)) * g.nx + gxw;
      const int node = j * W + wi;
#pragma unroll
      for (int f = 0; f < 11; ++f) fw[f * WP + node] = F[f * plane + go];
    }
  }
  if (DEPOSIT)
    for (int idx = threadIdx.x; idx < 3 * WP; idx += blockDim.x) jw[idx] = A(0);
  __syncthreads();

  using S = Spline<T, DEG>;
  const T dt = T(ph.dt), qs = T(ph.q) * T(g.inv_area);
  for (int k = threadIdx.x; k < it.z; k += blockDim.x) {
    const int64_t i = it.y + k;
    T x = p.x[i], y = p.y[i];
    T vx = p.v[0][i], vy = p.v[1][i], vz = p.v[2][i];
    if (GATHER) {
      T gv[11];
#pragma unroll
      for (int f = 0; f < 11; ++f) gv[f] = T(0);
      const T xi = x * T(g.inv_dx), eta = y * T(g.inv_dy);
      if (in_box(xi, eta, g)) {
        int sx, sy;
        T wx[S::NW], wy[S::NW];
        S::eval(xi, sx, wx);
        S::eval(eta, sy, wy);
        const int lx = (sx - ox) & (g.nx - 1), ly = (sy - oy) & (g.ny - 1);
        if (lx + DEG < W && ly + DEG < W) {
#pragma unroll
          for (int b = 0; b < S::NW; ++b) {
#pragma unroll
            for (int a = 0; a < S::NW; ++a) {
              const T w = wx[a] * wy[b];
              const T* nd = fw + (ly + b) * W + lx + a;
#pragma unroll
              for (int f = 0; f < 11; ++f) gv[f] += w * nd[f * WP];
            }
          }
        } else {
          gather_global<T, DEG>(sx, sy, wx, wy, F, g, gv);
        }
      }
      T Px = p.P[0][i], Py = p.P[1][i];
      const T Pz = p.P[2][i];
      const T wx0 = p.w[0][i], wy0 = p.w[1][i], wz0 = p.w[2][i];
      T nvx, nvy, nvz;
      push_one<T>(gv, Px, Py, Pz, vx, vy, vz, wx0, wy0, wz0, ph, nvx, nvy, nvz);
      p.P[0][i] = Px;
      p.P[1][i] = Py;
      p.w[0][i] = nvx;
      p.w[1][i] = nvy;
      p.w[2][i] = nvz;
      vx = nvx;
      vy = nvy;
      vz = nvz;
    }
    if (DEPOSIT) {
      x = wrapx<T>(x + vx * dt, T(g.lx));
      y = wrapx<T>(y + vy * dt, T(g.ly));
      p.x[i] = x;
      p.y[i] = y;
      const T xi = x * T(g.inv_dx), eta = y * T(g.inv_dy);
      if (in_box(xi, eta, g)) {
        int sx, sy;
        T wx[S::NW], wy[S::NW];
        S::eval(xi, sx, wx);
        S::eval(eta, sy, wy);
        const T jx = qs * vx, jy = qs * vy, jz = qs * vz;
        const int lx = (sx - ox) & (g.nx - 1), ly = (sy - oy) & (g.ny - 1);
        if (lx + DEG < W && ly + DEG < W) {
#pragma unroll
          for (int b = 0; b < S::NW; ++b) {
#pragma unroll
            for (int a = 0; a < S::NW; ++a) {
              const T w = wx[a] * wy[b];
              A* nd = jw + (ly + b) * W + lx + a;
              atomicAdd(nd, A(jx * w));
              atomicAdd(nd + WP, A(jy * w));
              atomicAdd(nd + 2 * WP, A(jz * w));
            }
          }
        } else {
          deposit_global<T, DEG>(sx, sy, wx, wy, jx, jy, jz, J, g);
        }
      }
    }
  }
  if (DEPOSIT) {
    __syncthreads();
    if (wi < W) {
      for (int j = wj0; j < W; j += wjs) {
        const size_t go = (size_t)((oy + j) & (g.ny - 1)) * g.nx + gxw;
        const int node = j * W + wi;
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          const A v = jw[c * WP + node];
          if (v != A(0)) atomicAdd(J + c * plane + go, (double)v);
        }
      }
    }
  }
}

template <typename T, int DEG, int MODE>
hipError_t launch_tiled_t(const InstDesc* D, int ninst, int nblocks, size_t lds, StepArgs sa, hipStream_t s) {
  hipFuncSetAttribute((const void*)k_tiled<T, DEG, MODE>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  hipLaunchKernelGGL((k_tiled<T, DEG, MODE>), dim3(nblocks), dim3(kThreads), lds, s, D, ninst, sa);
  return hipGetLastError();
}

template <typename T, int MODE>
hipError_t launch_tiled_deg(int degree, const InstDesc* D, int ninst, int nblocks, size_t lds, StepArgs sa,
                            hipStream_t s) {
  switch (degree) {
    case 1: return launch_tiled_t<T, 1, MODE>(D, ninst, nblocks, lds, sa, s);
    case 2: return launch_tiled_t<T, 2, MODE>(D, ninst, nblocks, lds, sa, s);
    default: return launch_tiled_t<T, 3, MODE>(D, ninst, nblocks, lds, sa, s);
  }
}

template <typename T>
hipError_t launch_tiled_mode(int mode, int degree, const InstDesc* D, int ninst, int nblocks, size_t lds,
                             StepArgs sa, hipStream_t s) {
  switch (mode) {
    case MODE_DEPOSIT: return launch_tiled_deg<T, MODE_DEPOSIT>(degree, D, ninst, nblocks, lds, sa, s);
    case MODE_GATHER_PUSH: return launch_tiled_deg<T, MODE_GATHER_PUSH>(degree, D, ninst, nblocks, lds, sa, s);
    default: return launch_tiled_deg<T, MODE_FUSED>(degree, D, ninst, nblocks, lds, sa, s);
  }
}

}  // namespace

size_t tiled_lds_bytes(int dtype, int mode, const TileP& tp) {
  const size_t es = dtype == PIC_F32 ? 4 : 8;
  return (mode != MODE_DEPOSIT ? (size_t)11 * tp.win_pad * es : 0) +
         (mode != MODE_GATHER_PUSH ? (size_t)3 * tp.win_pad * 8 : 0);
}
size_t sort_count_lds_bytes(const TileP& tp) { return (size_t)tp.ntiles * sizeof(int32_t); }
size_t sort_scatter_lds_bytes(const TileP& tp) { return (size_t)2 * tp.ntiles * sizeof(int32_t); }

// count (BK_COUNT blocks), scan (one block per instance), scatter (BK_PART blocks)
hipError_t launch_tile_sort(int dtype, const InstDesc* D, int ninst, int nb_count, int nb_part, size_t lds_count,
                            size_t lds_scatter, int src_set, hipStream_t s) {
  if (dtype == PIC_F32) {
    if (nb_count) hipLaunchKernelGGL(k_tile_count<float>, dim3(nb_count), dim3(kThreads), lds_count, s, D, ninst, src_set);
  } else {
    if (nb_count) hipLaunchKernelGGL(k_tile_count<double>, dim3(nb_count), dim3(kThreads), lds_count, s, D, ninst, src_set);
  }
  hipLaunchKernelGGL(k_tile_scan, dim3(ninst), dim3(1024), 0, s, D, ninst);
  if (dtype == PIC_F32) {
    if (nb_part) hipLaunchKernelGGL(k_tile_scatter<float>, dim3(nb_part), dim3(kThreads), lds_scatter, s, D, ninst, src_set);
  } else {
    if (nb_part) hipLaunchKernelGGL(k_tile_scatter<double>, dim3(nb_part), dim3(kThreads), lds_scatter, s, D, ninst, src_set);
  }
  return hipGetLastError();
}

hipError_t launch_tiled(int dtype, int mode, int degree, const InstDesc* D, int ninst, int nblocks, size_t lds,
                        StepArgs sa, hipStream_t s) {
  if (dtype == PIC_F32) return launch_tiled_mode<float>(mode, degree, D, ninst, nblocks, lds, sa, s);
  return launch_tiled_mode<double>(mode, degree, D, ninst, nblocks, lds, sa, s);
}

}  // namespace pic
