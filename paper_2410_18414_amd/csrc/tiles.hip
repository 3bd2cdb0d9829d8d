// Cell-sorted particle passes with LDS-privatised gather and deposition.
//
// The grid's cells are split into tiles of TS x TS cells.  Every few steps the
// particles are counting-sorted by cell, cells numbered tile-major
// (k_tile_count, k_cell_scan, k_tile_scatter): each tile's
// particles are contiguous and grouped by cell inside it.  The scan cuts each
// tile's range into chunks of at most CH particles, one chunk per workgroup.
//
// A workgroup owns a window of W x W mesh nodes around its tile: the tile's
// TS cells, a slack of S cells on each side (particles drift after the sort),
// and the widest stencil reach (one node below, two above the cell).  It
// copies the eleven gathered fields of the window into LDS, node-major (the
// node's fields in one 12-slot record, read as 16-byte vectors), gathers from
// there, accumulates its J contributions in an LDS window, and adds that
// window to the global float64 J with one atomic per non-zero node
// component.  A particle whose stencil leaves the window (it
// drifted further than S cells since the sort) takes the global-memory path
// for that operation, so results never depend on the sort.
//
// Consecutive lanes take consecutive particles, so the lanes of a wave mostly
// share a cell: the gather's LDS reads become broadcasts, and the deposit
// rotates each lane's stencil order so that lanes of one cell add to
// different LDS addresses at each atomic instruction.
//
// The per-particle arithmetic (spline weights, IAEM push, position update) is
// shared with the untiled kernels through particle_math.h.
#include "particle_math.h"

namespace pic {

namespace {

constexpr int kThreads = 256;
// slots per node of the LDS field window: the eleven gathered fields and one
// pad, so that a node's record is three 16-byte (float) or six (double) vectors
constexpr int kNodeSlots = kFieldSlots;
// fixed-point rounding by one FMA: 1.5 * 2^23 and its bit pattern
constexpr float kMagic = 12582912.0f;
constexpr uint32_t kMagicBits = 0x4B400000u;
constexpr uint64_t kMagicPair = ((uint64_t)kMagicBits << 32) | kMagicBits;

__device__ __forceinline__ void load_node(const float* p, float* q) {
  const float4* v = reinterpret_cast<const float4*>(p);
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    const float4 t = v[i];
    q[4 * i] = t.x;
    q[4 * i + 1] = t.y;
    q[4 * i + 2] = t.z;
    q[4 * i + 3] = t.w;
  }
}
__device__ __forceinline__ void load_node(const double* p, double* q) {
  const double2* v = reinterpret_cast<const double2*>(p);
#pragma unroll
  for (int i = 0; i < 6; ++i) {
    const double2 t = v[i];
    q[2 * i] = t.x;
    q[2 * i + 1] = t.y;
  }
}

// deterministic deposit's fallback for a stencil outside the window: each
// contribution rounded at the instance's fixed scale (float32: the window's
// one-FMA rounding; float64: llrint of the scaled product) and added to the
// int64 J planes
template <typename T, int DEG>
__device__ __forceinline__ void deposit_global_fixed(int sx, int sy, const T* wx, const T* wy, T sjx, T sjy, T sjz,
                                                     double* __restrict__ J, const GridP& g) {
  using S = Spline<T, DEG>;
  const size_t plane = (size_t)g.nx * g.ny;
  const gptr<unsigned long long> Jq = gp(reinterpret_cast<unsigned long long*>(J));
  auto q = [](T v, T w) -> long long {
    if constexpr (sizeof(T) == 4)
      return (long long)(int32_t)(__float_as_uint(__builtin_fmaf(v, w, kMagic)) - kMagicBits);
    else
      return llrint(v * w);
  };
#pragma unroll
  for (int b = 0; b < S::NW; ++b) {
    const size_t row = (size_t)wrapi(sy + b, g.ny) * g.nx;
#pragma unroll
    for (int a = 0; a < S::NW; ++a) {
      const T w = wx[a] * wy[b];
      const size_t o = row + wrapi(sx + a, g.nx);
      gadd(Jq + o, (unsigned long long)q(sjx, w));
      gadd(Jq + plane + o, (unsigned long long)q(sjy, w));
      gadd(Jq + 2 * plane + o, (unsigned long long)q(sjz, w));
    }
  }
}

// cell key of a position (cells floor(xi), clamped into the grid), numbered
// tile-major: tile * ts^2 + (row in tile) * ts + (column in tile)
__device__ __forceinline__ int cell_of(float xi, float eta, const TileP& tp) {
  int cx = (int)floorf(xi), cy = (int)floorf(eta);
  cx = cx < 0 ? 0 : (cx >= tp.nx ? tp.nx - 1 : cx);
  cy = cy < 0 ? 0 : (cy >= tp.ny ? tp.ny - 1 : cy);
  const int tile = (cy >> tp.log_ts) * tp.ntx + (cx >> tp.log_ts);
  const int m = tp.ts - 1;
  return (tile << (2 * tp.log_ts)) + ((cy & m) << tp.log_ts) + (cx & m);
}

template <typename T>
__device__ __forceinline__ int cell_key(T x, T y, const GridP& g, const TileP& tp) {
  const float xi = (float)(x * T(g.inv_dx)), eta = (float)(y * T(g.inv_dy));
  const bool ok = xi == xi && eta == eta;  // non-finite positions go to cell 0
  return ok ? cell_of(xi, eta, tp) : 0;
}

// The lanes of this lane's wave that hold the same key (0 for an inactive
// lane): a ballot per distinct key of the wave (particles are nearly sorted
// between sorts, so a wave holds few keys).
__device__ __forceinline__ uint64_t key_group(int key, bool active) {
  uint64_t pending = __ballot(active), mine = 0;
  while (pending) {
    const int leader = __ffsll((unsigned long long)pending) - 1;
    const int k0 = __shfl(key, leader);
    const uint64_t grp = __ballot(active && key == k0);
    if (active && key == k0) mine = grp;
    pending &= ~grp;
  }
  return mine;
}

// counters[key] += (lanes with this key): one atomic per distinct key of the
// wave, all issued by one instruction (the lowest lane of each group).
// Returns the counter's old value (the group's base) and the lane's rank in
// its group; with RET false the atomics return nothing and base is 0.
template <bool RET>
__device__ __forceinline__ int wave_group_add(int32_t* __restrict__ counters, int key, bool active, int& rank) {
  const int lane = threadIdx.x & 63;
  const uint64_t grp = key_group(key, active);
  const int leader = grp ? __ffsll((unsigned long long)grp) - 1 : lane;
  rank = __popcll(grp & ((1ull << lane) - 1ull));
  int b = 0;
  if (active && lane == leader) {
    const gptr<int32_t> ctr = gp(counters) + key;
    if (RET)
      b = __hip_atomic_fetch_add(ctr, (int32_t)__popcll(grp), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    else
      gadd(ctr, (int32_t)__popcll(grp));
  }
  return RET ? __shfl(b, leader) : 0;
}

// Cell histogram of the current positions: each block counts 1024 particles
// of one instance (flattened over instances, BK_COUNT), one atomic lane per
// distinct cell of a wave (particles stay nearly sorted).  The counter's old
// value plus the lane's rank in its wave group is the particle's slot among
// its cell's particles, kept for the scatter.
template <typename T>
__global__ void __launch_bounds__(kThreads) k_tile_count(const InstDesc* __restrict__ D, int ninst, int set) {
  const int ii = find_inst(D, ninst, BK_COUNT, blockIdx.x);
  const InstDesc& d = D[ii];
  const TileP tp = d.tp;
  const GridP g = d.g;
  const gptr<const T> px = gp((const T*)d.set[set][0]);
  const gptr<const T> py = gp((const T*)d.set[set][1]);
  const gptr<int32_t> rank = gp(d.tb.rank);
  const int64_t base = (int64_t)(blockIdx.x - d.blk[BK_COUNT]) * 1024;
  for (int k = 0; k < 4; ++k) {  // whole waves stay in the loop
    const int64_t i = base + k * kThreads + threadIdx.x;
    const bool act = i < d.n;
    const int c = act ? cell_key(px[i], py[i], g, tp) : 0;
    int r;
    const int base = wave_group_add<true>(d.tb.ccount, c, act, r);
    if (act) rank[i] = base + r;
  }
}

// Tile starts and the chunk list from the tile totals (one block, all of its
// threads): exclusive scan in passes of blockDim tiles.  The totals were
// written by other blocks of the same launch: read them device-coherently.
__device__ void tile_scan_block(const InstDesc& d, const TileP& tp) {
  __shared__ int32_t s_cnt[kThreads], s_chk[kThreads];
  __shared__ int32_t carry_p, carry_c;
  const int tid = threadIdx.x;
  if (tid == 0) {
    carry_p = 0;
    carry_c = 0;
  }
  __syncthreads();
  for (int base = 0; base < tp.ntiles; base += kThreads) {
    const int t = base + tid;
    const int c = t < tp.ntiles ? __hip_atomic_load(&d.tb.count[t], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) : 0;
    const int k = (c + tp.chunk - 1) / tp.chunk;
    s_cnt[tid] = c;
    s_chk[tid] = k;
    __syncthreads();
    // Hillis-Steele inclusive scans
    for (int off = 1; off < kThreads; off <<= 1) {
      const int a = tid >= off ? s_cnt[tid - off] : 0;
      const int b = tid >= off ? s_chk[tid - off] : 0;
      __syncthreads();
      s_cnt[tid] += a;
      s_chk[tid] += b;
      __syncthreads();
    }
    const int p0 = carry_p + s_cnt[tid] - c;  // exclusive
    const int k0 = carry_c + s_chk[tid] - k;
    if (t < tp.ntiles) {
      d.tb.start[t] = p0;
      d.tb.cstart[t] = k0;
      for (int j = 0; j < k; ++j) {
        const int s = p0 + j * tp.chunk;
        const int e = min(p0 + c, s + tp.chunk);
        d.tb.work[k0 + j] = make_int4(t, s, e - s, 0);
      }
    }
    __syncthreads();
    if (tid == kThreads - 1) {
      carry_p += s_cnt[kThreads - 1];
      carry_c += s_chk[kThreads - 1];
    }
    __syncthreads();
  }
  if (tid == 0) {
    d.tb.start[tp.ntiles] = carry_p;
    *d.tb.nwork = carry_c;
  }
}

// Cell cursors and tile starts (flattened over instances, BK_TILES: four tiles
// per block, one wave per tile).  A wave scans its tile's ts^2 cell counts
// into offsets from the tile's first slot (the scatter's cursors) and writes
// the tile's total; the block of the instance that finishes last (a
// device-scope counter, reset by that block) then scans the tile totals into
// tile starts and the chunk list.
__global__ void __launch_bounds__(kThreads) k_cell_scan(const InstDesc* __restrict__ D, int ninst) {
  const int ii = find_inst(D, ninst, BK_TILES, blockIdx.x);
  const InstDesc& d = D[ii];
  const TileP tp = d.tp;
  const int t = (blockIdx.x - d.blk[BK_TILES]) * (kThreads / 64) + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (t < tp.ntiles) {
    const int cells = tp.ts * tp.ts;
    int32_t* __restrict__ cc = d.tb.ccount + (size_t)t * cells;
    int32_t* __restrict__ cu = d.tb.ccursor + (size_t)t * cells;
    int run = 0;
    for (int j0 = 0; j0 < cells; j0 += 64) {
      const int j = j0 + lane;
      const int c = j < cells ? cc[j] : 0;
      int v = c;  // inclusive wave scan
      for (int off = 1; off < 64; off <<= 1) {
        const int u = __shfl_up(v, off);
        if (lane >= off) v += u;
      }
      if (j < cells) {
        cu[j] = run + v - c;
        cc[j] = 0;  // ready for the next sort
      }
      run += __shfl(v, 63);
    }
    if (lane == 0) d.tb.count[t] = run;
  }
  __shared__ int last;
  __threadfence();  // this block's totals are visible before it is counted
  __syncthreads();
  if (threadIdx.x == 0) {
    const int nb = (tp.ntiles + kThreads / 64 - 1) / (kThreads / 64);  // blocks of this instance
    last = atomicAdd(d.tb.done, 1) == nb - 1;
  }
  __syncthreads();
  if (!last) return;
  __threadfence();
  tile_scan_block(d, tp);
  if (threadIdx.x == 0) *d.tb.done = 0;  // ready for the next sort
}

// scatter set `src` into set `src ^ 1`, grouped by cell: particle i goes to its
// tile's start + its cell's offset in the tile + its slot in the cell (from the
// count pass); no atomics, so the copy streams.  The source is in the previous
// sort's cell order, so an XCD-contiguous run of source blocks covers one
// region of the grid, and the short runs its waves write per destination cell
// mostly land in that region: neighbouring runs of one cache line are then
// written through the same L2 rather than from several XCDs.
template <typename T>
__global__ void __launch_bounds__(kThreads) k_tile_scatter(const InstDesc* __restrict__ D, int ninst, int src) {
  const int bb = xcd_contiguous(blockIdx.x, gridDim.x);
  const int ii = find_inst(D, ninst, BK_PART, bb);
  const InstDesc& d = D[ii];
  const TileP tp = d.tp;
  const int64_t i = (int64_t)(bb - d.blk[BK_PART]) * kThreads + threadIdx.x;
  if (i >= d.n) return;  // no cross-lane operations below
  const void* const* S = d.set[src];
  void* const* Dd = d.set[src ^ 1];
  T rec[11];
#pragma unroll
  for (int a = 0; a < 11; ++a) rec[a] = gp((const T*)S[a])[i];
  const int32_t id = gp(d.ids[src])[i], slot = gp(d.tb.rank)[i];
  const int c = cell_key(rec[0], rec[1], d.g, tp);  // the count pass's key of the same positions
  const int tt = c >> (2 * tp.log_ts);
  const gptr<const int32_t> start = gp((const int32_t*)d.tb.start);
  const int32_t t0 = start[tt];
  const int rel = gp((const int32_t*)d.tb.ccursor)[c] + slot;  // slot in the tile
  const int64_t o = (int64_t)t0 + rel;
#pragma unroll
  for (int a = 0; a < 11; ++a) gp((T*)Dd[a])[o] = rec[a];
  gp(d.ids[src ^ 1])[o] = id;
  // a chunk's first and last particles record its span of cell rows (slots
  // are in cell order, cells row-major in the tile) for the tiled pass's
  // field-window rows; the cell scan wrote the field as zero
  const int j = rel / tp.chunk, in_chunk = rel - j * tp.chunk;
  const bool first = in_chunk == 0;
  const bool last = in_chunk == tp.chunk - 1 || rel == start[tt + 1] - t0 - 1;
  if (first || last) {
    const int row = (c & ((1 << (2 * tp.log_ts)) - 1)) >> tp.log_ts;
    const gptr<int> rows = gp(reinterpret_cast<int*>(d.tb.work + d.tb.cstart[tt] + j) + 3);
    if (first) __hip_atomic_fetch_or(rows, row, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (last) __hip_atomic_fetch_or(rows, row << 16, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
}

// ---------------------------------------------------------------------------
// the tiled particle pass

enum { MODE_DEPOSIT = 0, MODE_GATHER_PUSH = 1, MODE_FUSED = 2 };

// LDS storage unit of the deposit window: 8 bytes for both particle
// precisions.  Float64 particles add float64 values (on gfx950 the LDS float64
// add sustains many times the rate of the float32 add, which serialises per
// lane); float32 particles reuse the storage for the packed fixed-point sums.
template <typename T>
struct Acc {
  using type = double;
};

template <typename T, int DEG, int MODE, int TS, int SL>
__global__ void __launch_bounds__(kThreads) k_tiled(const InstDesc* __restrict__ D, int ninst, StepArgs sa) {
  constexpr bool GATHER = MODE != MODE_DEPOSIT;
  constexpr bool DEPOSIT = MODE != MODE_GATHER_PUSH;
  constexpr bool FIXEDPT = sizeof(T) == 4;  // fixed-point window (float32 particles)
  constexpr bool FIXED = TS > 0;
  using G = Geo<(FIXED ? TS : 1), (FIXED ? SL : 0)>;
  using A = typename Acc<T>::type;
  const int ii = find_inst(D, ninst, BK_WORK, blockIdx.x);
  const InstDesc& d = D[ii];
  const int item = blockIdx.x - d.blk[BK_WORK];
  if (item >= *gp(d.tb.nwork)) return;
  const i32x4 itv = *reinterpret_cast<gptr<const i32x4>>(gp(d.tb.work + item));
  const int4 it = make_int4(itv.x, itv.y, itv.z, itv.w);
  const GridP g = d.g;
  const PhysP ph = d.ph;
  const TileP tp = d.tp;
  // the chunk's particles from its first one on: lane offsets stay 32-bit
  const GParts<T> p = parts_from(global_parts(make_parts<T>(d, sa.cur, sa.vflip)), it.y);
  const T* __restrict__ F = GATHER ? (d.F32 ? (const T*)(const void*)d.F32 : (const T*)(const void*)d.F64) : nullptr;
  const gptr<const T> Fg = gp(F);
  // sub-stepped DIRK stage (deposit-only passes): deposit at x + c_i dt v into
  // J planes 3i..3i+2; only the last stage writes x^{n+1}
  const bool staged = !GATHER && sa.stage >= 0;
  double* __restrict__ J = d.J + (staged ? (size_t)3 * sa.stage * d.g.nx * d.g.ny : 0);
  const gptr<double> Jg = gp(J);
  const int W = FIXED ? G::W : tp.win;
  const int WP = FIXED ? G::WP : tp.win_pad;  // plane stride of the J window planes
  const int WF = field_pitch(W, (int)sizeof(T));  // row pitch of the field window
  const int FWN = field_window_nodes(W, (int)sizeof(T));  // its nodes
  // plane stride of the float64 J window: WP + 8 puts the three components of
  // a node 16 banks apart (WP itself is a multiple of the 64-bank cycle)
  const int JWP = WP + 8;
  const int ts = FIXED ? TS : tp.ts, slack = FIXED ? SL : tp.slack;
  // node indices modulo the grid: masks on power-of-two grids (the only ones
  // the fixed-geometry kernels run on), otherwise remainders; tiles of a grid
  // side that is not a multiple of the tile edge are partial at the high end
  const bool pw = FIXED || tp.pow2;
  auto modn = [&](int v, int n) { return pw ? (v & (n - 1)) : ((v % n) + n) % n; };
  // a stencil origin relative to the window origin: in [-n, 2n) because the
  // slack is below n - 1 (validated for grids that are not powers of two)
  auto modw = [&](int v, int n) { return pw ? (v & (n - 1)) : (v < 0 ? v + n : (v >= n ? v - n : v)); };
  const int tiy = pw ? it.x >> tp.log_ntx : it.x / tp.ntx, tix = it.x - tiy * tp.ntx;
  const int ox = tix * ts - slack - 1, oy = tiy * ts - slack - 1;
  // field-window rows this chunk can read: its particles' cell rows at the
  // sort lie in [r0, r1] (tile-local), they have moved at most the slack since
  // (the sort interval keeps them there), and a stencil of any degree starts
  // at most two nodes below its cell and spans at most six; a stencil outside
  // [jlo, jhi) takes the global gather, so the bound is a speed-up only
  const int jlo = max(0, (it.w & 0xffff) - 1), jhi = min(W, (it.w >> 16) + 2 * slack + 5);
  extern __shared__ __align__(16) unsigned char smem[];
  T* fw = reinterpret_cast<T*>(smem);
  A* jw = reinterpret_cast<A*>(smem + (GATHER ? (size_t)kNodeSlots * FWN * sizeof(T) : 0));
  const size_t plane = (size_t)g.nx * g.ny;
  // One particle per lane, consecutive lanes on consecutive particles.  The
  // set is sorted by cell, so the lanes of a wave mostly share one or two
  // cells: their gather reads hit the same LDS addresses (broadcasts).
  const int lane = threadIdx.x & 63;
  T cx = T(0), cy = T(0), cvx = T(0), cvy = T(0), cvz = T(0), cP[3] = {T(0), T(0), T(0)},
    cw[3] = {T(0), T(0), T(0)};
  // J carries v* = 2 v - v_prev: the deposit needs the older velocity too
  const bool jv = d.jvstar != 0;
  const bool det = d.det != 0;  // deterministic deposit: int64 J at the instance's fixed scale
  auto load = [&](uint32_t k) {
    cx = elt(p.x, k);
    cy = elt(p.y, k);
    cvx = elt(p.v[0], k);
    cvy = elt(p.v[1], k);
    cvz = elt(p.v[2], k);
    if (GATHER) {
#pragma unroll
      for (int c = 0; c < 3; ++c) cP[c] = elt(p.P[c], k);
    }
    if (GATHER || jv) {
#pragma unroll
      for (int c = 0; c < 3; ++c) cw[c] = elt(p.w[c], k);
    }
  };
  // the first particle's inputs are in flight while the window loads
  if ((int)threadIdx.x < it.z) load(threadIdx.x);
  // window sweeps without integer division: lanes of a row-group cover x
  // (row_lanes >= W, a power of two), row-groups cover y
  const int rl = FIXED ? G::RL : tp.row_lanes, lrl = FIXED ? G::LRL : tp.log_row_lanes;
  const int wi = threadIdx.x & (rl - 1), wj0 = threadIdx.x >> lrl, wjs = blockDim.x >> lrl;
  const int gxw = modn(ox + wi, g.nx);
  if (GATHER && wi < W) {
    if constexpr (sizeof(T) == 4) {
      // float32 fields are node-major in global memory as in LDS: a node is
      // three 16-byte vectors
      auto copy_row = [&](int j) {
        const size_t go = (size_t)modn(oy + j, g.ny) * g.nx + gxw;
        const gptr<const f32x4> src = reinterpret_cast<gptr<const f32x4>>(Fg + go * kFieldSlots);
        f32x4* dst = reinterpret_cast<f32x4*>(fw + (j * WF + wi) * kNodeSlots);
        const f32x4 a0 = src[0], a1 = src[1], a2 = src[2];
        dst[0] = a0;
        dst[1] = a1;
        dst[2] = a2;
      };
      if (FIXED) {
        constexpr int NJ = (G::W + (kThreads >> G::LRL) - 1) / (kThreads >> G::LRL);
#pragma unroll
        for (int r = 0; r < NJ; ++r) {
          const int j = wj0 + r * wjs;
          if (j >= jlo && j < jhi) copy_row(j);
        }
      } else {
        for (int j = wj0; j < W; j += wjs)
          if (j >= jlo && j < jhi) copy_row(j);
      }
    } else if (FIXED) {
      // compile-time sweep: a thread's rows (at most NJ) and fields all load
      // before the first LDS store
      constexpr int NJ = (G::W + (kThreads >> G::LRL) - 1) / (kThreads >> G::LRL);
      T v[NJ][11];
#pragma unroll
      for (int r = 0; r < NJ; ++r) {
        const int j = wj0 + r * wjs;
        if (j >= jlo && j < jhi) {
          const size_t go = (size_t)modn(oy + j, g.ny) * g.nx + gxw;
#pragma unroll
          for (int f = 0; f < 11; ++f) v[r][f] = Fg[f * plane + go];
        }
      }
#pragma unroll
      for (int r = 0; r < NJ; ++r) {
        const int j = wj0 + r * wjs;
        if (j >= jlo && j < jhi) {
#pragma unroll
          for (int f = 0; f < 11; ++f) fw[(j * WF + wi) * kNodeSlots + f] = v[r][f];
        }
      }
    } else {
      for (int j = wj0; j < W; j += wjs) {
        if (j < jlo || j >= jhi) continue;
        const size_t go = (size_t)modn(oy + j, g.ny) * g.nx + gxw;
        const int node = j * WF + wi;
#pragma unroll
        for (int f = 0; f < 11; ++f) fw[node * kNodeSlots + f] = Fg[f * plane + go];
      }
    }
  }
  // the naive charge deposit: rho^{n+1} from the same spline at x^{n+1}, a
  // fourth window plane flushed to the fourth J plane
  const bool naive = d.naive != 0;
  if (DEPOSIT) {
    // float64 window: 3 (naive: 4) planes of float64; fixed-point window
    // (float32 particles): JWP 64-bit x/y pairs then JWP 32-bit z values (and
    // JWP 32-bit rho values)
    const int nzero = sizeof(T) == 4 ? (naive ? 2 * JWP : (3 * JWP + 1) / 2) : (naive ? 4 : 3) * JWP;
    for (int idx = threadIdx.x; idx < nzero; idx += blockDim.x) jw[idx] = A(0);
  }
  __syncthreads();

  using S = Spline<T, DEG>;
  constexpr int NW = S::NW;
  // the spline weights are evaluated times S::kUnit (eval_unit): their products
  // carry kUnit^2, which the charge factors of the deposit and of the push
  // take back
  const T dt = T(ph.dt), qs = T(ph.q * g.inv_area / (S::kUnit * S::kUnit));
  PhysP phu = ph;
  phu.q = ph.q / (S::kUnit * S::kUnit);
  // Float32 particles deposit in fixed point: J_x and J_y as one packed pair
  // of int32 in a 64-bit integer atomic, J_z in a 32-bit one (two LDS atomics
  // per node instead of three float64 ones).  The scale is a power of two
  // 2^e chosen per chunk: every contribution is bounded by B = |q| c max(w) /
  // (dx dy) (|v| < c; 3c for |2 v - v_prev|), and B 2^qe0 < 2^30 (qe0 from the
  // host, d.qe0), so with e = qe0 - max(ceil(log2 count), 9) a node's sum over
  // the chunk stays below 2^30 (each packed half decodes for |sum| < 2^31) and
  // a single contribution below 2^21 (the rounding FMA needs below 2^22).
  unsigned long long* jxy_w = reinterpret_cast<unsigned long long*>(jw);     // [JWP]
  uint32_t* jz_w = reinterpret_cast<uint32_t*>(jw + JWP);                      // [JWP]
  uint32_t* jr_w = jz_w + JWP;                                                  // [JWP] (naive)
  float qscale = 1.0f;
  double inv_qscale = 1.0;
  if (FIXEDPT) {
    const int lz = it.z > 1 ? 32 - __clz(it.z - 1) : 0;  // ceil(log2 count)
    // deterministic deposit: the instance's fixed scale (that of a full chunk)
    int e = det ? d.qe_det : d.qe0 - (lz > 9 ? lz : 9);
    e = e > 100 ? 100 : (e < -100 ? -100 : e);  // a normal float scale, whatever q, c and the cell area
    qscale = __int_as_float((e + 127) << 23);
    inv_qscale = __longlong_as_double((long long)(1023 - e) << 52);
  }
  for (int k0 = 0; k0 < it.z; k0 += blockDim.x) {
    const int k = k0 + threadIdx.x;
    const bool act = k < it.z;
    T x = cx, y = cy, vx = cvx, vy = cvy, vz = cvz;
    T Px = cP[0], Py = cP[1], Pz = cP[2], w0 = cw[0], w1 = cw[1], w2 = cw[2];
    if (k + (int)blockDim.x < it.z) load(k + blockDim.x);  // next particle, in flight meanwhile
    if (GATHER && act) {
      T gv[11];
#pragma unroll
      for (int f = 0; f < 11; ++f) gv[f] = T(0);
      const T xi = x * T(g.inv_dx), eta = y * T(g.inv_dy);
      if (in_box(xi, eta, g)) {
        int sx, sy;
        T wx[NW], wy[NW];
        S::eval_unit(xi, sx, wx);
        S::eval_unit(eta, sy, wy);
        const int lx = modw(sx - ox, g.nx), ly = modw(sy - oy, g.ny);
        if (lx + DEG < W && ly >= jlo && ly + DEG < jhi) {
          const T* nd0 = fw + (ly * WF + lx) * kNodeSlots;
#pragma unroll
          for (int b = 0; b < NW; ++b) {
#pragma unroll
            for (int a = 0; a < NW; ++a) {
              const T w = wx[a] * wy[b];
              T q[kNodeSlots];
              load_node(nd0 + (b * WF + a) * kNodeSlots, q);
#pragma unroll
              for (int f = 0; f < 11; ++f) gv[f] += w * q[f];
            }
          }
        } else {
          gather_global<T, DEG>(sx, sy, wx, wy, F, g, gv);
        }
      }
      T nvx, nvy, nvz;
      push_one<T>(gv, Px, Py, Pz, vx, vy, vz, w0, w1, w2, phu, nvx, nvy, nvz);
      elt(p.P[0], k) = Px;
      elt(p.P[1], k) = Py;
      elt(p.w[0], k) = nvx;
      elt(p.w[1], k) = nvy;
      elt(p.w[2], k) = nvz;
      w0 = vx;
      w1 = vy;
      w2 = vz;
      vx = nvx;
      vy = nvy;
      vz = nvz;
    }
    if (DEPOSIT) {
      // set by an active lane; read only where inw, which an inactive lane
      // leaves false (no zero-initialisation for every particle)
      bool inw = false;
      int sx, sy, lx, ly;
      T wx[NW], wy[NW];
      T jx, jy, jz;
      if (act) {
        if (staged) {
          if (sa.stage == d.sc.stages - 1) {
            elt(p.x, k) = wrapx<T>(x + vx * dt, T(g.lx));
            elt(p.y, k) = wrapx<T>(y + vy * dt, T(g.ly));
          }
          const T sdt = T(ph.dt * d.sc.dirkC[sa.stage]);
          x = wrapx<T>(x + vx * sdt, T(g.lx));
          y = wrapx<T>(y + vy * sdt, T(g.ly));
        } else {
          x = wrapx<T>(x + vx * dt, T(g.lx));
          y = wrapx<T>(y + vy * dt, T(g.ly));
          elt(p.x, k) = x;
          elt(p.y, k) = y;
        }
        // a particle outside the box (not finite, or never wrapped) deposits
        // zero current with zero weights at a stand-in position inside it: no
        // branch around the deposit's set-up, whose zero-initialised values
        // would cost more than the selects
        const T xi0 = x * T(g.inv_dx), eta0 = y * T(g.inv_dy);
        const bool box = in_box(xi0, eta0, g);
        const T xi = box ? xi0 : T(0.5), eta = box ? eta0 : T(0.5);
        {
          S::eval_unit(xi, sx, wx);
          S::eval_unit(eta, sy, wy);
#pragma unroll
          for (int a = 0; a < NW; ++a) wx[a] = box ? wx[a] : T(0);
          if (jv) {
            jx = qs * (T(2) * vx - w0);
            jy = qs * (T(2) * vy - w1);
            jz = qs * (T(2) * vz - w2);
          } else {
            jx = qs * vx;
            jy = qs * vy;
            jz = qs * vz;
          }
          jx = box ? jx : T(0);
          jy = box ? jy : T(0);
          jz = box ? jz : T(0);
          lx = modw(sx - ox, g.nx);
          ly = modw(sy - oy, g.ny);
          inw = lx + DEG < W && ly + DEG < W;
          if (!inw) {
            if (det) {
              const T sc = FIXEDPT ? T(qscale) : T(d.det_scale);
              deposit_global_fixed<T, DEG>(sx, sy, wx, wy, jx * sc, jy * sc, jz * sc, J, g);
            } else {
              deposit_global<T, DEG>(sx, sy, wx, wy, jx, jy, jz, J, g);
              if (naive) {
#pragma unroll
                for (int b = 0; b < NW; ++b) {
                  const size_t row = (size_t)wrapi(sy + b, g.ny) * g.nx;
#pragma unroll
                  for (int a = 0; a < NW; ++a)
                    gadd(Jg + 3 * plane + row + wrapi(sx + a, g.nx), (double)(qs * (wx[a] * wy[b])));
                }
              }
            }
          }
        }
      }
      if (inw) {
        // per-lane rotation of stencil columns and rows: at step (a, b) lane l
        // adds to the stencil node whose absolute indices are congruent to
        // (a + l, b + l / NW) modulo NW (a stencil holds one node of every
        // residue pair), so two lanes can meet on one window address only when
        // their lane indices agree modulo NW^2 -- at most 64 / NW^2 lanes per
        // address, whatever cells the wave's particles are in (a rotation by
        // lane index alone lets lanes of neighbouring cells collide)
        const int ra = ((lane - sx) % NW + NW) % NW, rb = ((lane / NW - sy) % NW + NW) % NW;
        T wxr[NW], wyr[NW];
        int roff[NW], cxy[NW], cz[NW];  // rotated row offsets (nodes), column offsets (bytes)
#pragma unroll
        for (int t = 0; t < NW; ++t) {
          int ia = t + ra, ib = t + rb;
          ia = ia >= NW ? ia - NW : ia;
          ib = ib >= NW ? ib - NW : ib;
          wxr[t] = wx[t];
          wyr[t] = wy[t];
          roff[t] = ib * W;
          cxy[t] = ia * (int)sizeof(unsigned long long);
          cz[t] = ia * (int)sizeof(uint32_t);
        }
        rotate_lanes<NW>(wxr, ra);
        rotate_lanes<NW>(wyr, rb);
        // one packed x/y atomic and one z atomic per node, the same order in
        // every lane (a lane-dependent slot order splits the wave into two
        // halves that each issue both atomics)
        if constexpr (FIXEDPT) {
          const T sjx = jx * qscale, sjy = jy * qscale, sjz = jz * qscale, sjr = qs * qscale;
          if (inw) {
            const int base = ly * W + lx;
#pragma unroll
            for (int b = 0; b < NW; ++b) {
              unsigned char* xy_row = reinterpret_cast<unsigned char*>(jxy_w + base + roff[b]);
              unsigned char* z_row = reinterpret_cast<unsigned char*>(jz_w + base + roff[b]);
#pragma unroll
              for (int a = 0; a < NW; ++a) {
                const T w = wxr[a] * wyr[b];
                // the exact product rounded to the nearest integer, ties to
                // even (unbiased at the exact halves that scaled float32
                // products often are), in one FMA: for |s w| < 2^22 the sum
                // s w + 1.5 * 2^23 has unit spacing, so its bits are
                // kMagicBits + round(s w)
                const uint32_t bx = __float_as_uint(__builtin_fmaf(sjx, w, kMagic));
                const uint32_t by = __float_as_uint(__builtin_fmaf(sjy, w, kMagic));
                const uint32_t bz = __float_as_uint(__builtin_fmaf(sjz, w, kMagic));
                // (int64) ix + 2^32 (int64) iy modulo 2^64, ix = bx - kMagicBits, iy = by - kMagicBits
                const uint64_t pk = (((uint64_t)by << 32) | bx) - kMagicPair;
                atomicAdd(reinterpret_cast<unsigned long long*>(xy_row + cxy[a]), (unsigned long long)pk);
                atomicAdd(reinterpret_cast<uint32_t*>(z_row + cz[a]), bz - kMagicBits);
              }
            }
            // the naive charge plane in a loop of its own: a test inside the
            // node loop above costs every node two instructions
            if (naive) {
#pragma unroll
              for (int b = 0; b < NW; ++b) {
                unsigned char* r_row = reinterpret_cast<unsigned char*>(jr_w + base + roff[b]);
#pragma unroll
                for (int a = 0; a < NW; ++a) {
                  const uint32_t br = __float_as_uint(__builtin_fmaf(sjr, wxr[a] * wyr[b], kMagic));
                  atomicAdd(reinterpret_cast<uint32_t*>(r_row + cz[a]), br - kMagicBits);
                }
              }
            }
          }
        } else if (inw && det) {
          // deterministic deposit (float64): int64 window sums of the products
          // rounded at the instance's fixed scale
          unsigned long long* nq0 = reinterpret_cast<unsigned long long*>(jw) + ly * W + lx;
          const T dx_ = jx * T(d.det_scale), dy_ = jy * T(d.det_scale), dz_ = jz * T(d.det_scale);
#pragma unroll
          for (int b = 0; b < NW; ++b) {
            unsigned char* row = reinterpret_cast<unsigned char*>(nq0 + roff[b]);
#pragma unroll
            for (int a = 0; a < NW; ++a) {
              const T w = wxr[a] * wyr[b];
              unsigned long long* nq = reinterpret_cast<unsigned long long*>(row + cxy[a]);
              atomicAdd(nq, (unsigned long long)llrint(dx_ * w));
              atomicAdd(nq + JWP, (unsigned long long)llrint(dy_ * w));
              atomicAdd(nq + 2 * JWP, (unsigned long long)llrint(dz_ * w));
            }
          }
        } else if (inw) {
          // float64 window: float64 LDS atomics
          A* nd0 = jw + ly * W + lx;
#pragma unroll
          for (int b = 0; b < NW; ++b) {
            unsigned char* row = reinterpret_cast<unsigned char*>(nd0 + roff[b]);
#pragma unroll
            for (int a = 0; a < NW; ++a) {
              const T w = wxr[a] * wyr[b];
              A* nd = reinterpret_cast<A*>(row + cxy[a]);
              atomicAdd(nd, A(jx * w));
              atomicAdd(nd + JWP, A(jy * w));
              atomicAdd(nd + 2 * JWP, A(jz * w));
              if (naive) atomicAdd(nd + 3 * JWP, A(qs * w));
            }
          }
        }
      }
    }
  }
  if (DEPOSIT) {
    __syncthreads();
    if (wi < W) {
      for (int j = wj0; j < W; j += wjs) {
        const size_t go = (size_t)modn(oy + j, g.ny) * g.nx + gxw;
        const int node = j * W + wi;
        if (FIXEDPT) {
          const uint64_t v = jxy_w[node];
          const int32_t X = (int32_t)(uint32_t)v;
          const int32_t Y = (int32_t)((int64_t)(v - (uint64_t)(int64_t)X) >> 32);
          const int32_t Z = (int32_t)jz_w[node];
          if (det) {  // int64 J planes at the same fixed scale: exact, order-free sums
            const gptr<unsigned long long> Jq = gp(reinterpret_cast<unsigned long long*>(J));
            if (X) gadd(Jq + go, (unsigned long long)(long long)X);
            if (Y) gadd(Jq + plane + go, (unsigned long long)(long long)Y);
            if (Z) gadd(Jq + 2 * plane + go, (unsigned long long)(long long)Z);
          } else {
            if (X) gadd(Jg + go, X * inv_qscale);
            if (Y) gadd(Jg + plane + go, Y * inv_qscale);
            if (Z) gadd(Jg + 2 * plane + go, Z * inv_qscale);
            if (naive) {
              const int32_t R = (int32_t)jr_w[node];
              if (R) gadd(Jg + 3 * plane + go, R * inv_qscale);
            }
          }
        } else if (det) {
          const unsigned long long* jq = reinterpret_cast<const unsigned long long*>(jw);
          const gptr<unsigned long long> Jq = gp(reinterpret_cast<unsigned long long*>(J));
#pragma unroll
          for (int c = 0; c < 3; ++c) {
            const unsigned long long v = jq[c * JWP + node];
            if (v) gadd(Jq + c * plane + go, v);
          }
        } else {
          const int nc = naive ? 4 : 3;
          for (int c = 0; c < nc; ++c) {
            const A v = jw[c * JWP + node];
            if (v != A(0)) gadd(Jg + c * plane + go, (double)v);
          }
        }
      }
    }
  }
}

// compiled window geometries: geo 0 = from TileP, 1 = 16x16 tiles with slack
// 3, 2 = 8x8 tiles with slack 3
template <typename T, int DEG, int MODE>
hipError_t launch_tiled_t(int geo, const InstDesc* D, int ninst, int nblocks, size_t lds, StepArgs sa,
                          hipStream_t s) {
  const void* fn = geo == 1 ? (const void*)k_tiled<T, DEG, MODE, 16, 3>
                   : geo == 2 ? (const void*)k_tiled<T, DEG, MODE, 8, 3>
                              : (const void*)k_tiled<T, DEG, MODE, 0, 0>;
  (void)hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (geo == 1)
    hipLaunchKernelGGL((k_tiled<T, DEG, MODE, 16, 3>), dim3(nblocks), dim3(kThreads), lds, s, D, ninst, sa);
  else if (geo == 2)
    hipLaunchKernelGGL((k_tiled<T, DEG, MODE, 8, 3>), dim3(nblocks), dim3(kThreads), lds, s, D, ninst, sa);
  else
    hipLaunchKernelGGL((k_tiled<T, DEG, MODE, 0, 0>), dim3(nblocks), dim3(kThreads), lds, s, D, ninst, sa);
  return hipGetLastError();
}

template <typename T, int MODE>
hipError_t launch_tiled_deg(int degree, int geo, const InstDesc* D, int ninst, int nblocks, size_t lds, StepArgs sa,
                            hipStream_t s) {
  switch (degree) {
    case 1: return launch_tiled_t<T, 1, MODE>(geo, D, ninst, nblocks, lds, sa, s);
    case 2: return launch_tiled_t<T, 2, MODE>(geo, D, ninst, nblocks, lds, sa, s);
    case 4: return launch_tiled_t<T, 4, MODE>(geo, D, ninst, nblocks, lds, sa, s);
    case 5: return launch_tiled_t<T, 5, MODE>(geo, D, ninst, nblocks, lds, sa, s);
    default: return launch_tiled_t<T, 3, MODE>(geo, D, ninst, nblocks, lds, sa, s);
  }
}

template <typename T>
hipError_t launch_tiled_mode(int mode, int degree, int geo, const InstDesc* D, int ninst, int nblocks, size_t lds,
                             StepArgs sa, hipStream_t s) {
  switch (mode) {
    case MODE_DEPOSIT: return launch_tiled_deg<T, MODE_DEPOSIT>(degree, geo, D, ninst, nblocks, lds, sa, s);
    case MODE_GATHER_PUSH: return launch_tiled_deg<T, MODE_GATHER_PUSH>(degree, geo, D, ninst, nblocks, lds, sa, s);
    default: return launch_tiled_deg<T, MODE_FUSED>(degree, geo, D, ninst, nblocks, lds, sa, s);
  }
}

}  // namespace

size_t tiled_lds_bytes(int dtype, int mode, const TileP& tp, bool naive) {
  const size_t es = dtype == PIC_F32 ? 4 : 8;
  // J window bytes per node: float32 a packed x/y pair, z (and rho) in 32
  // bits; float64 three (four) planes
  const size_t jb = dtype == PIC_F32 ? (naive ? 16 : 12) : (naive ? 32 : 24);
  return (mode != MODE_DEPOSIT ? (size_t)kNodeSlots * field_window_nodes(tp.win, (int)es) * es : 0) +
         (mode != MODE_GATHER_PUSH ? jb * (tp.win_pad + 8) + 8 : 0);
}

// count (BK_COUNT blocks), cell scan with the tile scan in its last block
// per instance (BK_TILES blocks), scatter (BK_PART blocks)
hipError_t launch_tile_sort(int dtype, const InstDesc* D, int ninst, int nb_count, int nb_tiles, int nb_part,
                            int src_set, hipStream_t s) {
  if (nb_count) {
    if (dtype == PIC_F32)
      hipLaunchKernelGGL(k_tile_count<float>, dim3(nb_count), dim3(kThreads), 0, s, D, ninst, src_set);
    else
      hipLaunchKernelGGL(k_tile_count<double>, dim3(nb_count), dim3(kThreads), 0, s, D, ninst, src_set);
  }
  hipLaunchKernelGGL(k_cell_scan, dim3(nb_tiles), dim3(kThreads), 0, s, D, ninst);
  if (nb_part) {
    if (dtype == PIC_F32)
      hipLaunchKernelGGL(k_tile_scatter<float>, dim3(nb_part), dim3(kThreads), 0, s, D, ninst, src_set);
    else
      hipLaunchKernelGGL(k_tile_scatter<double>, dim3(nb_part), dim3(kThreads), 0, s, D, ninst, src_set);
  }
  return hipGetLastError();
}

int tiled_geometry(const TileP& tp) {
  if (!tp.pow2) return 0;  // the fixed geometries wrap node indices by masks
  if (tp.slack == 3 && tp.ts == 16) return 1;
  if (tp.slack == 3 && tp.ts == 8) return 2;
  return 0;
}

hipError_t launch_tiled(int dtype, int mode, int degree, int geo, const InstDesc* D, int ninst, int nblocks,
                        size_t lds, StepArgs sa, hipStream_t s) {
  if (dtype == PIC_F32) return launch_tiled_mode<float>(mode, degree, geo, D, ninst, nblocks, lds, sa, s);
  return launch_tiled_mode<double>(mode, degree, geo, D, ninst, nblocks, lds, sa, s);
}

}  // namespace pic
