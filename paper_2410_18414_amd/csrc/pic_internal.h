// Internal declarations shared by the libpic translation units.
//
// Every hot-path kernel runs over a flattened grid that covers all instances
// of a context (one instance for the plain API, many for an ensemble): each
// instance owns a contiguous range of blocks, found by binary search over the
// per-instance block offsets in its descriptor (InstDesc, device memory).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>

#include "pic.h"

namespace pic {

// ---------------------------------------------------------------------------
// geometry / physics

struct GridP {
  int nx, ny, nxh;          // nxh = nx/2 + 1
  double lx, ly, dx, dy;
  double inv_dx, inv_dy, inv_area;
};

struct PhysP {
  double dt, q, m, c;
};

// Row pitch (in nodes) of the tiled pass's LDS field window of W x W nodes.
// A float32 node record is 12 dwords, so at one gather instruction two lanes
// whose stencils start at nodes n1, n2 read the same bank group when
// 12 (n1 - n2) = 0 mod 64, i.e. n1 - n2 = 0 mod 16; with row pitch P,
// n1 - n2 = P dy + dx for the lanes' cell offset (dx, dy).  As the cell order
// ages between sorts a wave's particles spread over neighbouring cells, and
// every offset on that lattice adds conflicts (the pitch W = 25 of 16-cell
// tiles puts (2, -2) on it, W = 17 of 8-cell tiles (1, -1)).  The pitch is the
// one of W .. W + 7 whose lattice points with |dx|, |dy| <= 3 weigh least
// (weight 1 / (dx^2 + dy^2)), among those that keep the fused pass's
// workgroups per CU (160 KB of LDS with the float32 J window beside the field
// window).
// Float64 records (24 dwords) keep the pitch W.
__host__ __device__ constexpr double pitch_conflicts(int P) {
  double wgt = 0.0;
  for (int dy = -3; dy <= 3; ++dy)
    for (int dx = -3; dx <= 3; ++dx)
      if ((dx != 0 || dy != 0) && (P * dy + dx) % 16 == 0) wgt += 1.0 / (dx * dx + dy * dy);
  return wgt;
}
__host__ __device__ constexpr long fused_lds_f32(int W, int P) {
  return 48L * W * P + 12L * ((W * W + 63) / 64 * 64 + 8) + 8;
}
// workgroups per CU the LDS admits, counted up to 4 (the register file holds
// about four of the fused pass's 256-thread workgroups)
__host__ __device__ constexpr long fused_wgs(int W, int P) {
  return 163840L / fused_lds_f32(W, P) < 4 ? 163840L / fused_lds_f32(W, P) : 4;
}
__host__ __device__ constexpr int field_pitch(int W, int es) {
  if (es != 4) return W;
  int best = W;
  double bw = pitch_conflicts(W);
  for (int P = W + 1; P < W + 8; ++P) {
    if (fused_wgs(W, P) < fused_wgs(W, W)) continue;
    const double wgt = pitch_conflicts(P);
    if (wgt < bw) {
      bw = wgt;
      best = P;
    }
  }
  return best;
}
// nodes of the field window: W rows of the pitch (float64: padded to 64 nodes)
__host__ __device__ constexpr int field_window_nodes(int W, int es) {
  return es == 4 ? W * field_pitch(W, es) : (W * W + 63) / 64 * 64;
}

// Particle SoA pointers.  v[0..2] = v^n, w[0..2] = v^{n-1} (overwritten with v^{n+1}).
template <typename T>
struct Parts {
  T* x;
  T* y;
  T* P[3];
  T* v[3];
  T* w[3];
  int32_t* id;
};

// Device pointers into global memory.  A pointer the compiler reads from a
// descriptor in memory is generic to it, and generic (flat) loads and stores
// count against the LDS wait counter as well as the vector-memory one: a wave
// that waits for its LDS reads would then also wait for every global load it
// has in flight (e.g. the next particle's prefetch).  Kernels cast such
// pointers into the global address space before using them.
template <typename T>
using gptr = __attribute__((address_space(1))) T*;
template <typename T>
__device__ __forceinline__ gptr<T> gp(T* p) {
  return (gptr<T>)p;
}
// relaxed device-scope atomic add through a global pointer
template <typename T>
__device__ __forceinline__ void gadd(gptr<T> p, T v) {
  __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// A complex128 array in global memory.  Elements are read and written through
// their two float64 parts (HIP's vector classes cannot be loaded or stored
// through address-space pointers); the compiler merges each pair into one
// 16-byte access.
struct GC2Ref {
  gptr<double> p;
  __device__ __forceinline__ operator double2() const { return make_double2(p[0], p[1]); }
  __device__ __forceinline__ const GC2Ref& operator=(const double2& v) const {
    p[0] = v.x;
    p[1] = v.y;
    return *this;
  }
};
struct GC2 {
  gptr<double> p;
  __device__ __forceinline__ GC2Ref operator[](size_t i) const { return GC2Ref{p + 2 * i}; }
};
__device__ __forceinline__ GC2 gc2(const double2* a) {
  return GC2{gp(const_cast<double*>(reinterpret_cast<const double*>(a)))};
}
// 16 bytes of global memory as four floats or ints (a compiler vector type)
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef int i32x4 __attribute__((ext_vector_type(4)));

// Particle SoA pointers in the global address space (device code)
template <typename T>
struct GParts {
  gptr<T> x;
  gptr<T> y;
  gptr<T> P[3];
  gptr<T> v[3];
  gptr<T> w[3];
  gptr<int32_t> id;
};

// element k of a global array whose base b is wave-uniform: the byte offset
// stays 32-bit, so the access is one global instruction with the base in
// scalar registers and the offset in a vector register
template <typename T>
__device__ __forceinline__ __attribute__((address_space(1))) T& elt(gptr<T> b, uint32_t k) {
  return *(gptr<T>)((__attribute__((address_space(1))) char*)b + k * (uint32_t)sizeof(T));
}

// k with its relation to the previous iteration hidden from the loop
// optimiser: in a loop over particles, every elt() access then stays scalar
// base + 32-bit offset instead of becoming a per-lane 64-bit pointer carried
// around the loop (two VGPRs per array)
__device__ __forceinline__ uint32_t opaque_index(uint32_t k) {
  asm volatile("" : "+v"(k));
  return k;
}

// XCD-contiguous block order: the dispatcher deals consecutive workgroups to
// the eight XCDs in turn (block b to XCD b mod 8); this bijection of [0, nb)
// gives each XCD one contiguous run of logical blocks instead of every eighth,
// so that neighbouring logical blocks share one L2
__device__ __forceinline__ int xcd_contiguous(int b, int nb) {
  const int q = nb >> 3, r = nb & 7, x = b & 7, j = b >> 3;
  return x * q + min(x, r) + j;
}

template <typename T>
__device__ __forceinline__ GParts<T> global_parts(const Parts<T>& p) {
  GParts<T> g;
  g.x = gp(p.x);
  g.y = gp(p.y);
  for (int c = 0; c < 3; ++c) {
    g.P[c] = gp(p.P[c]);
    g.v[c] = gp(p.v[c]);
    g.w[c] = gp(p.w[c]);
  }
  g.id = gp(p.id);
  return g;
}

// the same arrays from particle `first` on (first is the same for the whole
// workgroup, so the new bases stay in scalar registers)
template <typename T>
__device__ __forceinline__ GParts<T> parts_from(GParts<T> g, int64_t first) {
  g.x += first;
  g.y += first;
  for (int c = 0; c < 3; ++c) {
    g.P[c] += first;
    g.v[c] += first;
    g.w[c] += first;
  }
  g.id += first;
  return g;
}

// Spectral history slot table for one update: slot index of each (group, level).
struct HistSlots {
  int rho[6];
  int rho_new;
  int phi[12];
  int phi_new;
  int A[12];                // slot of component 0; components are +1, +2
  int A_new;
  int vphi, vA, J[2], J_new;
};

// Tile decomposition for the sorted particle passes (tiles.hip)
struct TileP {
  int nx, ny;      // mesh nodes
  int ts;          // tile edge in cells
  int ntx, nty, ntiles;  // ceil(n / ts): the last tile of a row or column may be partial
  int log_ts, log_ntx;
  int slack;       // cells a particle may drift after the sort and stay in the window
  int win;         // window edge in nodes: ts + 2*slack + 3
  int win_pad;     // win*win rounded up to a multiple of 64 (LDS plane stride)
  int row_lanes;   // power of two >= win: threads per window row in the sweeps
  int log_row_lanes;
  int chunk;       // max particles per workgroup
  int max_work;    // ntiles + ceil(capacity/chunk): bound on the chunk count
  int pow2;        // 1: nx and ny are powers of two (node indices wrap by masks)
};

// Window geometry: compile-time for the compiled tile shapes (TS > 0: tiles of
// TS x TS cells, slack SL), so that every window offset of the gather and the
// deposit is an immediate of the LDS instruction; TS = 0 reads it from TileP.
template <int TS, int SL>
struct Geo {
  static constexpr int W = TS + 2 * SL + 3;
  static constexpr int WP = (W * W + 63) / 64 * 64;
  static constexpr int RL = W <= 8 ? 8 : (W <= 16 ? 16 : (W <= 32 ? 32 : 64));
  static constexpr int LRL = RL == 8 ? 3 : (RL == 16 ? 4 : (RL == 32 ? 5 : 6));
};

// Particles are counting-sorted by cell, cells numbered tile-major (the
// ts*ts cells of tile t are keys t*ts*ts .. (t+1)*ts*ts - 1), so each tile's
// particles are contiguous and, inside the tile, grouped by cell.
struct TileBufs {
  int32_t* count;    // [ntiles]   particles per tile (written by the cell scan)
  int32_t* start;    // [ntiles+1] first particle of each tile
  int32_t* ccount;   // [ntiles*ts*ts] particles per cell key; zero between sorts
  int32_t* ccursor;  // [ntiles*ts*ts] first slot of each cell, from its tile's start
  int4* work;        // [max_work] (tile, first particle, count, rows): rows = r0 | r1 << 16, the
                     //            tile-local cell rows of the chunk's first and last particle at the sort
  int32_t* cstart;   // [ntiles]   each tile's first chunk in work
  int32_t* nwork;    // [1]        chunks in use
  int32_t* done;     // [1]        blocks of the cell scan finished; zero between sorts
  int32_t* rank;     // [capacity] each particle's slot among its cell's particles (count pass)
};

struct SchemeCoef {
  int scheme, k;            // scheme family (BDF, CDF2, DIRK2 = every DIRK); BDF order
  int form;                 // CDF2 family: 0 implicit, 1 semi-implicit, 2 explicit
  double a[7];              // BDF first-derivative coefficients (step dt)
  double Cn[13];            // C_i / C_0 of the twice-applied operator
  double inv_alpha2;        // 1/alpha^2 of the single Helmholtz solve (BDF, CDF-2)
  int stages;               // DIRK family: 2 or 3
  int substep;              // DIRK family: 1 = stage currents deposited per stage (PIC_FLAG_DIRK_SUBSTEP)
  double dirkA[3][3], dirkB[3], dirkC[3];
  double dt, c, eps0, mu0;
};

// Mesh fields for the gather: the float64 fields are planar F[12][ny][nx];
// the float32 copy (float32 particles) is node-major F[ny][nx][kFieldSlots]
// -- the eleven gathered fields and phi~ of a node form one 48-byte record
// (three 16-byte vectors), the layout of the tiled passes' LDS windows.
constexpr int kFieldSlots = 12;

// block ranges of the flattened kernels
enum BlockKind {
  BK_R2C = 0,    // (ny/R_r2c) x 3 blocks
  BK_COL = 1,    // nxh x columns_parts(scheme) blocks
  BK_C2R = 2,    // (ny/R_c2r) x 6 blocks
  BK_WORK = 3,   // tp.max_work blocks (tiled particle pass)
  BK_PART = 4,   // ceil(capacity/256) blocks (untiled passes, scatter)
  BK_COUNT = 5,  // ceil(capacity/1024) blocks (tile counting)
  BK_TILES = 6,  // ceil(ntiles/4) blocks (per-tile cell scan, one wave per tile)
  BK_NKINDS = 7
};

// One instance of the method: static for the life of a context.
struct InstDesc {
  GridP g;
  PhysP ph;
  TileP tp;
  SchemeCoef sc;
  void* set[2][11];         // particle arrays of the two sort sets: x, y, P(3), V0(3), V1(3)
  int32_t* ids[2];
  double* J;
  double2* T;
  double2* H;
  double2* U;
  double* F64;
  float* F32;
  const double2* twx;
  const double2* twy;
  double* LF;               // adjoint buffers (PIC_FLAG_ADJOINT, else null): [11][ny][nx] mesh-field adjoints,
  double2* LS;              // [11][nxh][ny] their x-transforms (planes 0..2 reused for the J adjoint columns),
  double* LJ;               // [3][ny][nx] adjoint of J,
  double* LAM;              // [11][capacity] the held particle adjoint in slot order, LAM2 its permutation buffer,
  double* LAM2;
  int32_t* LIDS;            // [capacity] the original particle of each LAM slot, LINV its inverse,
  int32_t* LINV;
  int32_t* LFLAG;           // set when the particle order differs from LIDS
  double* RB;               // naive charge deposit (PIC_FLAG_NAIVE_RHO, else null): [ny][nx] ion background
  int naive;                // 1: J holds a fourth plane, the deposited rho; T a fourth component
  int jvstar;               // 1: J carries v* = 2 v - v_prev (PIC_FLAG_JVSTAR)
  int qe0;                  // float32 fixed-point deposit: B 2^qe0 < 2^30 for the contribution bound B
  int det;                  // 1: deterministic deposit (PIC_FLAG_DETERMINISTIC): J planes hold int64 at scale 2^qe_det
  int qe_det;               // that scale's exponent (float32: every chunk's window scale too)
  double det_scale, det_unscale;  // 2^qe_det, 2^-qe_det
  TileBufs tb;
  int64_t n;                // particles loaded
  int R_r2c, R_c2r, nb_col; // rows per block of the row kernels; forward batch of the adjoint column kernel
  int blk[BK_NKINDS];       // first block of this instance in each flattened grid
};

// Per-launch state common to every instance of a context (instances advance in lockstep).
struct StepArgs {
  int cur;    // current particle set (0/1)
  int vflip;  // 0: V0 = v^n, V1 = v^{n-1}; 1: swapped
  int stage;  // deposit passes: -1 = x^{n+1} and J^{n+1}; i >= 0 = DIRK stage i of the
              // sub-stepped currents (deposit at x + c_i dt v into J planes 3i..3i+2;
              // the last stage also writes x^{n+1})
};

// real J planes of an instance: 3, a fourth (the naive mode's rho), or three per DIRK stage
__host__ __device__ inline int j_planes(const SchemeCoef& sc, int naive) {
  return sc.substep ? 3 * sc.stages : 3 + naive;
}

template <typename T>
__host__ __device__ inline Parts<T> make_parts(const InstDesc& d, int set, int vflip) {
  Parts<T> p;
  p.x = (T*)d.set[set][0];
  p.y = (T*)d.set[set][1];
  for (int c = 0; c < 3; ++c) p.P[c] = (T*)d.set[set][2 + c];
  const int vb = vflip ? 8 : 5, wb = vflip ? 5 : 8;
  for (int c = 0; c < 3; ++c) {
    p.v[c] = (T*)d.set[set][vb + c];
    p.w[c] = (T*)d.set[set][wb + c];
  }
  p.id = d.ids[set];
  return p;
}

// instance owning flattened block b of kind k: largest i with D[i].blk[k] <= b
__device__ __forceinline__ int find_inst(const InstDesc* __restrict__ D, int ninst, int kind, int b) {
  int lo = 0, hi = ninst - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (D[mid].blk[kind] <= b) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

// ---------------------------------------------------------------------------
// launchers (each returns hipGetLastError() of its launches)

hipError_t launch_fill_f64(double* p, size_t n, double v, hipStream_t s);
// s S(x_g - x_p) of the particles of `parts` (a Parts<float|double>) added to R
hipError_t launch_charge(int dtype, int degree, const void* parts, int64_t n, GridP g, double s, double* R,
                         hipStream_t st);

// particles.hip: untiled passes (flattened over instances) and per-instance I/O
// mode: 0 deposit (position update + deposit), 1 gather + push, 2 fused
hipError_t launch_untiled(int dtype, int mode, int degree, const InstDesc* D, int ninst, int nblocks, StepArgs sa,
                          hipStream_t s);
hipError_t launch_init_particles(int dtype, const void* parts, int64_t n, const double* x, const double* y,
                                 const double* P, GridP g, PhysP ph, hipStream_t s);
hipError_t launch_get_particles(int dtype, const void* parts, int64_t n, double* out, hipStream_t s);
// max(|v_x|, |v_y|) over the set as float bits, atomically maxed into *out (zeroed by the caller)
hipError_t launch_max_inplane(int dtype, const void* parts, int64_t n, uint32_t* out, hipStream_t s);
// deterministic deposit: the int64 J planes of an instance as float64 (J export)
hipError_t launch_j_export(const long long* src, double* dst, size_t n, double unscale, hipStream_t s);
hipError_t launch_set_particles(int dtype, const void* parts, int64_t n, const double* in, GridP g, hipStream_t s);
hipError_t launch_particle_diag(int dtype, const void* parts, int64_t n, PhysP ph, double* out2, hipStream_t s);

// tiles.hip
size_t tiled_lds_bytes(int dtype, int mode, const TileP& tp, bool naive);
hipError_t launch_tile_sort(int dtype, const InstDesc* D, int ninst, int nb_count, int nb_tiles, int nb_part,
                            int src_set, hipStream_t s);
// geometry code of a tile plan: a compiled window shape (1, 2) or 0 (from TileP)
int tiled_geometry(const TileP& tp);
hipError_t launch_tiled(int dtype, int mode, int degree, int geo, const InstDesc* D, int ninst, int nblocks,
                        size_t lds, StepArgs sa, hipStream_t s);

// field.hip
void fft_make_twiddles(int n, double* host_re_im);  // n complex entries
int rows_r2c_R(int nx, int ny);
int rows_c2r_R(int nx, int ny);
int columns_nb(int ny);
size_t rows_r2c_lds_bytes(int nx, int ny);
size_t rows_c2r_lds_bytes(int nx, int ny);
size_t adj_columns_lds_bytes(int ny);
// blocks per kx of the forward column kernel (4 for BDF-k and CDF-2, split
// by output; 1 for DIRK-2) and the split kernel's LDS bytes
int columns_parts(int scheme);
size_t columns_split_lds_bytes(int ny, int nstage);  // nstage: sub-stepped DIRK stages (else 0)
// adj = true: the adjoint field solve's transforms (LF -> LS, LS -> LJ; one instance)
hipError_t launch_rows_r2c(const InstDesc* D, int ninst, int nblocks, size_t lds, hipStream_t s, bool adj = false);
hipError_t launch_columns(int scheme, int bdf_order, const InstDesc* D, int ninst, int nblocks, size_t lds,
                          HistSlots hs, int max_ny, hipStream_t s);
// f64out: the float64 mesh planes too (float32 contexts skip them in the step)
hipError_t launch_rows_c2r(const InstDesc* D, int ninst, int nblocks, size_t lds, hipStream_t s, bool adj = false,
                           bool f64out = false);
hipError_t launch_hist_transpose(const double2* src, double2* dst, int nfield, GridP g, bool to_external,
                                 hipStream_t s);
// adjoint.hip (one float64 BDF-k instance; D[0])
hipError_t launch_adj_push(int degree, const InstDesc* D, int64_t n, StepArgs sa, double* lam, int64_t ls,
                           hipStream_t s);
hipError_t launch_adj_deposit(int degree, const InstDesc* D, int64_t n, StepArgs sa, double* lam, int64_t ls,
                              hipStream_t s);
hipError_t launch_lam_set(int64_t n, const double* src, double* LAM, int64_t ls, int32_t* LIDS, const int32_t* ids,
                          hipStream_t s);
hipError_t launch_lam_get(int64_t n, const double* LAM, int64_t ls, const int32_t* LIDS, double* dst, hipStream_t s);
hipError_t launch_lam_follow(int64_t n, const int32_t* ids, double* LAM, double* LAM2, int64_t ls, int32_t* LIDS,
                             int32_t* LINV, int32_t* flag, hipStream_t s);
// cell-sorted variants over the forward's chunks (push: mesh fields and their
// adjoints in LDS windows; deposit: lambda_J window)
size_t adj_tiled_lds_bytes(const TileP& tp, bool push);
hipError_t launch_adj_tiled(bool push, int degree, int geo, const InstDesc* D, int nblocks, size_t lds, StepArgs sa,
                            double* lam, int64_t ls, hipStream_t s);
hipError_t launch_adj_columns(int bdf_order, const InstDesc* D, int nxh, size_t lds, double* lam_hist, hipStream_t s);
hipError_t launch_adj_seed_energy(const double2* H, GridP g, SchemeCoef sc, HistSlots hs, double scale,
                                  double* lam_hist, int nf, hipStream_t s);
hipError_t launch_adj_initial(int64_t n, const double* P, PhysP ph, double* lam, hipStream_t s);

hipError_t launch_field_diag(const double2* H, GridP g, SchemeCoef sc, HistSlots hs, double* out, hipStream_t s);

}  // namespace pic
