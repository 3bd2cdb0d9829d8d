// Internal declarations shared by the libpic translation units.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>

#include "pic.h"

namespace pic {

// ---------------------------------------------------------------------------
// geometry / physics passed to kernels by value

struct GridP {
  int nx, ny, nxh;          // nxh = nx/2 + 1
  double lx, ly, dx, dy;
  double inv_dx, inv_dy, inv_area;
};

struct PhysP {
  double dt, q, m, c;
};

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

// Spectral history slot table for one update: slot index of each (group, level).
// Groups (per scheme) are documented in field.hip; up to 12 level entries.
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
  int ntx, nty, ntiles;
  int log_ts, log_ntx;
  int slack;       // cells a particle may drift after the sort and stay in the window
  int win;         // window edge in nodes: ts + 2*slack + 3
  int win_pad;     // win*win rounded up to a multiple of 64 (LDS plane stride)
  int row_lanes;   // power of two >= win: threads per window row in the sweeps
  int log_row_lanes;
  int chunk;       // max particles per workgroup
  int max_work;    // ntiles + ceil(capacity/chunk): bound on the chunk count
};

struct TileBufs {
  int32_t* key;     // [capacity] tile of each particle at the last sort
  int32_t* count;   // [ntiles]   zero between sorts
  int32_t* start;   // [ntiles+1] first particle of each tile
  int32_t* cursor;  // [ntiles]
  int4* work;       // [max_work] (tile, first particle, count, 0)
  int32_t* nwork;   // [1]        chunks in use
};

struct SchemeCoef {
  int scheme, k;            // scheme id; BDF order
  double a[7];              // BDF first-derivative coefficients (step dt)
  double Cn[13];            // C_i / C_0 of the twice-applied operator
  double inv_alpha2;        // 1/alpha^2 of the single Helmholtz solve (BDF, CDF-2)
  double dirkA[2][2], dirkB[2], dirkC[2];
  double dt, c, eps0, mu0;
};

// ---------------------------------------------------------------------------
// launchers (each returns hipGetLastError() of its launch)

hipError_t launch_fill_f64(double* p, size_t n, double v, hipStream_t s);

// particles.hip
hipError_t launch_init_particles(int dtype, void* parts, int64_t n, const double* x,
                                 const double* y, const double* P, GridP g, PhysP ph,
                                 hipStream_t s);
hipError_t launch_deposit(int dtype, int degree, const void* parts, int64_t n, double* J,
                          GridP g, PhysP ph, hipStream_t s);
hipError_t launch_gather_push(int dtype, int degree, const void* parts, int64_t n,
                              const void* F, GridP g, PhysP ph, hipStream_t s);
hipError_t launch_fused(int dtype, int degree, const void* parts, int64_t n, const void* F,
                        double* J, GridP g, PhysP ph, hipStream_t s);
hipError_t launch_get_particles(int dtype, const void* parts, int64_t n, double* out,
                                hipStream_t s);
hipError_t launch_set_particles(int dtype, void* parts, int64_t n, const double* in, GridP g,
                                hipStream_t s);
hipError_t launch_particle_diag(int dtype, const void* parts, int64_t n, PhysP ph,
                                double* out2, hipStream_t s);

// tiles.hip  (mode: 0 deposit, 1 gather+push, 2 fused)
size_t tiled_lds_bytes(int dtype, int mode, const TileP& tp);
hipError_t launch_tile_sort(int dtype, const void* src, void* dst, int64_t n, const TileBufs& tb, GridP g,
                            TileP tp, hipStream_t s);
hipError_t launch_tiled(int dtype, int mode, int degree, const void* parts, const TileBufs& tb, const void* F,
                        double* J, GridP g, PhysP ph, TileP tp, hipStream_t s);

// field.hip
size_t fft_twiddle_count(int n);
void fft_make_twiddles(int n, double* host_re_im);    // n complex entries
hipError_t launch_rows_r2c(double* J, double2* T, const double2* twx, GridP g, hipStream_t s);
size_t columns_lds_bytes(int ny);
hipError_t launch_columns(const double2* T, double2* H, double2* U, const double2* twy,
                          GridP g, SchemeCoef sc, HistSlots hs, hipStream_t s);
hipError_t launch_rows_c2r(const double2* U, double* F64, float* F32, const double2* twx,
                           GridP g, hipStream_t s);
hipError_t launch_hist_transpose(const double2* src, double2* dst, int nfield, GridP g,
                                 bool to_external, hipStream_t s);
hipError_t launch_field_diag(const double2* H, GridP g, SchemeCoef sc, HistSlots hs,
                             double* out, hipStream_t s);

}  // namespace pic
