// libpic C ABI: validation, workspace layout, phase state machine and launch
// sequencing of Algorithm 1 (arXiv 2410.18414, Sec. 4.2).
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "pic_internal.h"

using namespace pic;

namespace {

thread_local std::string g_err;

enum Phase { EMPTY = 0, READY = 1, DEPOSITED = 2, SOLVED = 3 };

constexpr size_t kAlign = 256;
inline size_t align_up(size_t v) { return (v + kAlign - 1) & ~(kAlign - 1); }
inline bool pow2(int v) { return v > 0 && (v & (v - 1)) == 0; }

struct Layout {
  size_t part_arrays;  // two particle sets, each 11 arrays (cap x es) + ids
  size_t set_bytes;    // bytes of one set
  size_t tkey, tcount, tstart, tcursor, twork, tnwork;
  size_t J, T, H, U, F64, F32, twx, twy, diag, total;
  size_t plane_c;      // complex entries per spectral plane
};

// History groups: ring sizes and slot bases.  A ring of R levels for a field
// of `width` components occupies R*width consecutive slots; level j of the
// history before update number s lives at ring position (s - j) mod R.
struct Ring {
  int base = 0, size = 1, width = 1;
  int slot(int64_t s, int level) const {
    const int r = (int)(((s - level) % size + size) % size);
    return base + r * width;
  }
};

struct Hist {
  Ring rho, phi, A, vphi, vA, J;
  int nslots = 0;
  int nexport = 0;
};

Hist plan_history(const pic_config_t& c) {
  Hist h;
  int b = 0;
  auto mk = [&](Ring& r, int size, int width) {
    r.base = b;
    r.size = size;
    r.width = width;
    b += size * width;
  };
  if (c.scheme == PIC_SCHEME_BDF) {
    const int k = c.bdf_order;
    mk(h.rho, k, 1);
    mk(h.phi, 2 * k, 1);
    mk(h.A, 2 * k, 3);
    h.nexport = k + 2 * k + 6 * k;
  } else if (c.scheme == PIC_SCHEME_CDF2) {
    mk(h.rho, 3, 1);
    mk(h.phi, 3, 1);
    mk(h.A, 2, 3);
    mk(h.J, 2, 3);
    h.nexport = 18;
  } else {
    mk(h.rho, 2, 1);
    mk(h.phi, 2, 1);
    mk(h.vphi, 1, 1);
    mk(h.A, 2, 3);
    mk(h.vA, 1, 3);
    mk(h.J, 1, 3);
    h.nexport = 17;
  }
  h.nslots = b;
  return h;
}

bool validate(const pic_config_t* c, std::string& msg) {
  if (!c) { msg = "cfg is NULL"; return false; }
  if (c->abi_version != PIC_ABI_VERSION) { msg = "abi_version mismatch"; return false; }
  if (!pow2(c->nx) || !pow2(c->ny) || c->nx < 8 || c->ny < 8 || c->nx > 1024 || c->ny > 1024) {
    msg = "nx, ny must be powers of two in [8, 1024]";
    return false;
  }
  if (!(c->lx > 0) || !(c->ly > 0) || !std::isfinite(c->lx) || !std::isfinite(c->ly)) {
    msg = "lx, ly must be positive and finite";
    return false;
  }
  if (c->spline_degree < 1 || c->spline_degree > 3) { msg = "spline_degree must be 1, 2 or 3"; return false; }
  if (c->scheme < PIC_SCHEME_BDF || c->scheme > PIC_SCHEME_DIRK2) { msg = "unknown scheme"; return false; }
  if (c->scheme == PIC_SCHEME_BDF && (c->bdf_order < 1 || c->bdf_order > 6)) {
    msg = "bdf_order must be 1..6";
    return false;
  }
  if (c->particle_dtype != PIC_F32 && c->particle_dtype != PIC_F64) { msg = "particle_dtype"; return false; }
  if (!(c->dt > 0) || !std::isfinite(c->dt)) { msg = "dt must be positive"; return false; }
  if (!(c->c > 0) || !(c->eps0 > 0) || !(c->mu0 > 0)) { msg = "c, eps0, mu0 must be positive"; return false; }
  if (std::fabs(c->c * c->c * c->eps0 * c->mu0 - 1.0) > 1e-12) {
    msg = "c^2 eps0 mu0 must equal 1";
    return false;
  }
  if (!std::isfinite(c->q) || !(c->m > 0) || !std::isfinite(c->m)) { msg = "q finite, m > 0 required"; return false; }
  if (c->dt * c->c >= c->lx || c->dt * c->c >= c->ly) {
    msg = "c dt must be below the box size (one wrap per step)";
    return false;
  }
  if (c->max_particles < 1 || c->max_particles > ((int64_t)1 << 31) - 1) {
    msg = "max_particles must be in [1, 2^31)";
    return false;
  }
  if (c->sort_interval < 0) { msg = "sort_interval must be >= 0"; return false; }
  if (c->tile_cells && (!pow2(c->tile_cells) || c->tile_cells < 4 || c->tile_cells > 64 ||
                        c->tile_cells > c->nx || c->tile_cells > c->ny)) {
    msg = "tile_cells must be 0 or a power of two in [4, 64] not above nx, ny";
    return false;
  }
  if (c->chunk && (c->chunk < 64 || c->chunk > 65536)) { msg = "chunk must be 0 or in [64, 65536]"; return false; }
  if (c->slack < 0 || c->slack > 8) { msg = "slack must be in [0, 8]"; return false; }
  for (int i = 0; i < 4; ++i)
    if (c->reserved[i]) { msg = "reserved fields must be zero"; return false; }
  return true;
}

// Tile plan: tiles of 16x16 cells (smaller on small grids), a slack of three
// cells, chunks of at most 1024 particles per workgroup, unless the config
// sets them.
TileP plan_tiles(const pic_config_t& c) {
  TileP t{};
  t.nx = c.nx;
  t.ny = c.ny;
  t.ts = c.tile_cells ? c.tile_cells : std::min(16, std::min(c.nx, c.ny));
  t.ntx = c.nx / t.ts;
  t.nty = c.ny / t.ts;
  t.ntiles = t.ntx * t.nty;
  t.log_ts = 0;
  while ((1 << t.log_ts) < t.ts) t.log_ts++;
  t.log_ntx = 0;
  while ((1 << t.log_ntx) < t.ntx) t.log_ntx++;
  t.slack = c.slack ? c.slack : 3;
  t.win = t.ts + 2 * t.slack + 3;
  t.win_pad = (t.win * t.win + 63) / 64 * 64;
  t.row_lanes = 1;
  t.log_row_lanes = 0;
  while (t.row_lanes < t.win) {
    t.row_lanes <<= 1;
    t.log_row_lanes += 1;
  }
  t.chunk = c.chunk ? c.chunk : 1024;
  t.max_work = t.ntiles + (int)((c.max_particles + t.chunk - 1) / t.chunk);
  return t;
}

Layout plan(const pic_config_t& c) {
  Layout L{};
  const size_t es = c.particle_dtype == PIC_F32 ? 4 : 8;
  const size_t cap = (size_t)c.max_particles;
  const size_t nxh = c.nx / 2 + 1;
  const size_t plane_r = (size_t)c.nx * c.ny;
  L.plane_c = nxh * c.ny;
  const Hist h = plan_history(c);
  size_t o = 0;
  auto take = [&](size_t bytes) {
    const size_t at = o;
    o = align_up(o + bytes);
    return at;
  };
  L.set_bytes = 11 * align_up(cap * es) + align_up(cap * 4);
  L.part_arrays = take(2 * L.set_bytes);
  const TileP tp = plan_tiles(c);
  L.tkey = take(cap * 4);
  L.tcount = take((size_t)tp.ntiles * 4);
  L.tstart = take(((size_t)tp.ntiles + 1) * 4);
  L.tcursor = take((size_t)tp.ntiles * 4);
  L.twork = take((size_t)tp.max_work * 16);
  L.tnwork = take(4);
  L.J = take(3 * plane_r * 8);
  L.T = take(3 * L.plane_c * 16);
  L.H = take((size_t)h.nslots * L.plane_c * 16);
  L.U = take(8 * L.plane_c * 16);
  L.F64 = take(12 * plane_r * 8);
  L.F32 = c.particle_dtype == PIC_F32 ? take(12 * plane_r * 4) : 0;
  L.twx = take((size_t)c.nx * 16);
  L.twy = take((size_t)c.ny * 16);
  L.diag = take((16 + 2 * 256) * 8);
  L.total = o;
  return L;
}

// BDF-k first-derivative coefficients by differentiating the Lagrange
// interpolant through t = 0, -1, ..., -k at t = 0 (unit step):
// a_0 = sum_{m=1}^k 1/m;  a_j = -(1/j) prod_{m != 0, j} m/(m - j).
void bdf_coefficients(int k, double* a) {
  a[0] = 0;
  for (int m = 1; m <= k; ++m) a[0] += 1.0 / m;
  for (int j = 1; j <= k; ++j) {
    double p = -1.0 / j;
    for (int m = 1; m <= k; ++m)
      if (m != j) p *= (double)m / (double)(m - j);
    a[j] = p;
  }
}

}  // namespace

struct pic_ctx_s {
  pic_config_t cfg{};
  hipStream_t stream = nullptr;
  char* ws = nullptr;
  Layout L{};
  Hist hist{};
  GridP g{};
  PhysP ph{};
  SchemeCoef sc{};
  int64_t n = 0;
  int64_t nupd = 0;  // completed field updates (history head)
  int vflip = 0;     // which velocity block holds v^n
  int cur = 0;       // which particle set is current
  TileP tp{};
  TileBufs tb{};
  bool sorted = false;   // tiled kernels in use (no PIC_FLAG_NO_SORT)
  int sort_every = 4;    // position updates between sorts
  int moves = 0;         // position updates since the last sort
  Phase phase = EMPTY;
  std::string err;
  int device = 0;

  // optional per-launch-group timing (pic_set_kernel_timing)
  bool timing = false;
  struct EvPair {
    hipEvent_t a = nullptr, b = nullptr;
    int cls = 0;
  };
  std::vector<EvPair> ev;  // pool; the first ev_used entries hold pending pairs
  size_t ev_used = 0;
  double t_ms[PIC_KCLASS_COUNT] = {0};
  double t_n[PIC_KCLASS_COUNT] = {0};

  ~pic_ctx_s() {
    for (auto& e : ev) {
      if (e.a) hipEventDestroy(e.a);
      if (e.b) hipEventDestroy(e.b);
    }
  }
  // fold pending pairs into the totals (synchronises the stream)
  hipError_t fold_timing() {
    if (!ev_used) return hipSuccess;
    hipError_t e = hipStreamSynchronize(stream);
    if (e != hipSuccess) return e;
    for (size_t i = 0; i < ev_used; ++i) {
      float ms = 0;
      e = hipEventElapsedTime(&ms, ev[i].a, ev[i].b);
      if (e != hipSuccess) return e;
      t_ms[ev[i].cls] += ms;
      t_n[ev[i].cls] += 1;
    }
    ev_used = 0;
    return hipSuccess;
  }
  // returns the pair to record around a launch of class cls, or nullptr
  EvPair* begin_timed(int cls) {
    if (!timing) return nullptr;
    if (ev_used == 4096 && fold_timing() != hipSuccess) return nullptr;
    if (ev_used == ev.size()) {
      EvPair p;
      if (hipEventCreate(&p.a) != hipSuccess || hipEventCreate(&p.b) != hipSuccess) return nullptr;
      ev.push_back(p);
    }
    EvPair* p = &ev[ev_used++];
    p->cls = cls;
    hipEventRecord(p->a, stream);
    return p;
  }
  void end_timed(EvPair* p) {
    if (p) hipEventRecord(p->b, stream);
  }

  int es() const { return cfg.particle_dtype == PIC_F32 ? 4 : 8; }
  size_t cap_bytes() const { return align_up((size_t)cfg.max_particles * es()); }
  char* arr(int k, int set) const { return ws + L.part_arrays + set * L.set_bytes + (size_t)k * cap_bytes(); }
  char* arr(int k) const { return arr(k, cur); }
  int32_t* ids(int set) const { return (int32_t*)arr(11, set); }
  double* J() const { return (double*)(ws + L.J); }
  double2* T() const { return (double2*)(ws + L.T); }
  double2* H() const { return (double2*)(ws + L.H); }
  double2* U() const { return (double2*)(ws + L.U); }
  double* F64() const { return (double*)(ws + L.F64); }
  float* F32() const { return cfg.particle_dtype == PIC_F32 ? (float*)(ws + L.F32) : nullptr; }
  const void* Fgather() const {
    return cfg.particle_dtype == PIC_F32 ? (const void*)F32() : (const void*)F64();
  }
  double2* twx() const { return (double2*)(ws + L.twx); }
  double2* twy() const { return (double2*)(ws + L.twy); }
  double* diag() const { return (double*)(ws + L.diag); }

  // particle pointer block in the layout of Parts<T> (same for float/double)
  template <typename T>
  Parts<T> parts_t(int set) const {
    Parts<T> p;
    p.x = (T*)arr(0, set);
    p.y = (T*)arr(1, set);
    for (int c = 0; c < 3; ++c) p.P[c] = (T*)arr(2 + c, set);
    const int vb = vflip ? 8 : 5, wb = vflip ? 5 : 8;
    for (int c = 0; c < 3; ++c) {
      p.v[c] = (T*)arr(vb + c, set);
      p.w[c] = (T*)arr(wb + c, set);
    }
    p.id = ids(set);
    return p;
  }
  // storage for either instantiation (identical layout of pointers)
  struct PartsAny {
    union {
      Parts<float> f;
      Parts<double> d;
    };
  };
  PartsAny parts(int set) const {
    PartsAny a;
    if (cfg.particle_dtype == PIC_F32) a.f = parts_t<float>(set);
    else a.d = parts_t<double>(set);
    return a;
  }
  PartsAny parts() const { return parts(cur); }

  HistSlots slots(int64_t s) const {
    HistSlots h{};
    const Hist& r = hist;
    for (int j = 0; j < r.rho.size && j < 6; ++j) h.rho[j] = r.rho.slot(s, j);
    h.rho_new = r.rho.slot(s + 1, 0);
    for (int j = 0; j < r.phi.size && j < 12; ++j) h.phi[j] = r.phi.slot(s, j);
    h.phi_new = r.phi.slot(s + 1, 0);
    for (int j = 0; j < r.A.size && j < 12; ++j) h.A[j] = r.A.slot(s, j);
    h.A_new = r.A.slot(s + 1, 0);
    h.vphi = r.vphi.base;
    h.vA = r.vA.base;
    for (int j = 0; j < r.J.size && j < 2; ++j) h.J[j] = r.J.slot(s, j);
    h.J_new = r.J.slot(s + 1, 0);
    return h;
  }

  pic_status_t fail(pic_status_t st, const std::string& m) {
    err = m;
    return st;
  }
  pic_status_t hip(hipError_t e, const char* what) {
    if (e == hipSuccess) return PIC_OK;
    err = std::string(what) + ": " + hipGetErrorString(e);
    return PIC_ERR_HIP;
  }
};

namespace {

// counting sort of the particles by tile into the other set
pic_status_t do_sort(pic_ctx_t c) {
  if (!c->sorted) return PIC_OK;
  auto src = c->parts(c->cur);
  auto dst = c->parts(c->cur ^ 1);
  auto* t = c->begin_timed(4);
  hipError_t e = launch_tile_sort(c->cfg.particle_dtype, &src, &dst, c->n, c->tb, c->g, c->tp, c->stream);
  c->end_timed(t);
  pic_status_t st = c->hip(e, "tile sort");
  if (st) return st;
  c->cur ^= 1;
  c->moves = 0;
  return PIC_OK;
}

// sort first when the next position update could carry a particle past the slack
pic_status_t maybe_sort(pic_ctx_t c) {
  if (c->sorted && c->moves >= c->sort_every) return do_sort(c);
  return PIC_OK;
}

pic_status_t do_deposit(pic_ctx_t c) {
  pic_status_t st = maybe_sort(c);
  if (st) return st;
  auto pa = c->parts();
  auto* t = c->begin_timed(0);
  hipError_t e = c->sorted ? launch_tiled(c->cfg.particle_dtype, 0, c->cfg.spline_degree, &pa, c->tb, nullptr,
                                          c->J(), c->g, c->ph, c->tp, c->stream)
                           : launch_deposit(c->cfg.particle_dtype, c->cfg.spline_degree, &pa, c->n, c->J(), c->g,
                                            c->ph, c->stream);
  c->end_timed(t);
  c->moves += 1;
  return c->hip(e, "deposit launch");
}

pic_status_t do_solve(pic_ctx_t c) {
  auto* t = c->begin_timed(1);
  pic_status_t st = c->hip(launch_rows_r2c(c->J(), c->T(), c->twx(), c->g, c->stream), "rows_r2c launch");
  if (st) return st;
  st = c->hip(launch_columns(c->T(), c->H(), c->U(), c->twy(), c->g, c->sc, c->slots(c->nupd), c->stream),
              "columns launch");
  if (st) return st;
  st = c->hip(launch_rows_c2r(c->U(), c->F64(), c->F32(), c->twx(), c->g, c->stream), "rows_c2r launch");
  c->end_timed(t);
  if (st) return st;
  c->nupd += 1;
  return PIC_OK;
}

pic_status_t do_gather_push(pic_ctx_t c, bool fused) {
  if (fused) {
    pic_status_t st = maybe_sort(c);
    if (st) return st;
  }
  auto pa = c->parts();
  auto* t = c->begin_timed(fused ? 3 : 2);
  hipError_t e;
  if (c->sorted)
    e = launch_tiled(c->cfg.particle_dtype, fused ? 2 : 1, c->cfg.spline_degree, &pa, c->tb, c->Fgather(), c->J(),
                     c->g, c->ph, c->tp, c->stream);
  else
    e = fused ? launch_fused(c->cfg.particle_dtype, c->cfg.spline_degree, &pa, c->n, c->Fgather(), c->J(), c->g,
                             c->ph, c->stream)
              : launch_gather_push(c->cfg.particle_dtype, c->cfg.spline_degree, &pa, c->n, c->Fgather(), c->g,
                                   c->ph, c->stream);
  c->end_timed(t);
  if (fused) c->moves += 1;
  pic_status_t st = c->hip(e, fused ? "fused launch" : "gather_push launch");
  if (st) return st;
  c->vflip ^= 1;  // v^{n+1} was written over v^{n-1}
  return PIC_OK;
}

pic_status_t reset_fields(pic_ctx_t c) {
  pic_status_t st = c->hip(launch_fill_f64((double*)c->H(), (size_t)c->hist.nslots * c->L.plane_c * 2, 0.0,
                                           c->stream),
                           "history fill");
  if (st) return st;
  st = c->hip(launch_fill_f64(c->J(), (size_t)3 * c->cfg.nx * c->cfg.ny, 0.0, c->stream), "J fill");
  if (st) return st;
  c->nupd = 0;
  return PIC_OK;
}

}  // namespace

namespace {
// external history order (see pic.h) as a list of internal slots
std::vector<int> export_slots(pic_ctx_t c) {
  std::vector<int> v;
  const Hist& h = c->hist;
  const int64_t s = c->nupd;
  auto ring = [&](const Ring& r, int levels) {
    for (int j = 0; j < levels; ++j)
      for (int w = 0; w < r.width; ++w) v.push_back(r.slot(s, j) + w);
  };
  ring(h.rho, h.rho.size);
  ring(h.phi, h.phi.size);
  if (c->cfg.scheme == PIC_SCHEME_DIRK2) ring(h.vphi, 1);
  ring(h.A, h.A.size);
  if (c->cfg.scheme == PIC_SCHEME_DIRK2) ring(h.vA, 1);
  if (c->cfg.scheme != PIC_SCHEME_BDF) ring(h.J, h.J.size);
  return v;
}

pic_status_t history_io(pic_ctx_t c, double* ext, bool to_external) {
  const std::vector<int> slots = export_slots(c);
  const size_t plane = c->L.plane_c;
  for (size_t f = 0; f < slots.size(); ++f) {
    double2* in_slot = c->H() + (size_t)slots[f] * plane;
    double2* ext_f = (double2*)ext + f * plane;
    hipError_t e = to_external ? launch_hist_transpose(in_slot, ext_f, 1, c->g, true, c->stream)
                               : launch_hist_transpose(ext_f, in_slot, 1, c->g, false, c->stream);
    if (e != hipSuccess) return c->hip(e, "history transpose");
  }
  return PIC_OK;
}
}  // namespace

extern "C" {

size_t pic_workspace_bytes(const pic_config_t* cfg) {
  std::string m;
  if (!validate(cfg, m)) {
    g_err = m;
    return 0;
  }
  return plan(*cfg).total;
}

int32_t pic_history_fields(const pic_config_t* cfg) {
  std::string m;
  if (!validate(cfg, m)) {
    g_err = m;
    return -1;
  }
  return plan_history(*cfg).nexport;
}

const char* pic_last_error(pic_ctx_t ctx) { return ctx ? ctx->err.c_str() : g_err.c_str(); }

pic_status_t pic_create(const pic_config_t* cfg, void* workspace, size_t ws_bytes, void* hip_stream,
                        pic_ctx_t* out) {
  std::string m;
  if (!out) {
    g_err = "out is NULL";
    return PIC_ERR_INVALID_ARG;
  }
  *out = nullptr;
  if (!validate(cfg, m)) {
    g_err = m;
    return PIC_ERR_INVALID_ARG;
  }
  const Layout L = plan(*cfg);
  if (!workspace || ((uintptr_t)workspace & (kAlign - 1))) {
    g_err = "workspace must be a 256-byte aligned device pointer";
    return PIC_ERR_WORKSPACE;
  }
  if (ws_bytes < L.total) {
    g_err = "workspace too small: need " + std::to_string(L.total) + " bytes";
    return PIC_ERR_WORKSPACE;
  }
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) {
    g_err = "hipGetDevice failed";
    return PIC_ERR_HIP;
  }
  int max_lds = 0;
  hipDeviceGetAttribute(&max_lds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev);
  if (columns_lds_bytes(cfg->ny) > (size_t)max_lds) {
    g_err = "ny too large for this device's LDS";
    return PIC_ERR_UNSUPPORTED;
  }
  auto* c = new pic_ctx_s();
  c->cfg = *cfg;
  c->stream = (hipStream_t)hip_stream;
  c->ws = (char*)workspace;
  c->L = L;
  c->hist = plan_history(*cfg);
  c->device = dev;
  GridP& g = c->g;
  g.nx = cfg->nx;
  g.ny = cfg->ny;
  g.nxh = cfg->nx / 2 + 1;
  g.lx = cfg->lx;
  g.ly = cfg->ly;
  g.dx = cfg->lx / cfg->nx;
  g.dy = cfg->ly / cfg->ny;
  g.inv_dx = 1.0 / g.dx;
  g.inv_dy = 1.0 / g.dy;
  g.inv_area = 1.0 / (g.dx * g.dy);
  c->ph = PhysP{cfg->dt, cfg->q, cfg->m, cfg->c};
  c->tp = plan_tiles(*cfg);
  c->tb.key = (int32_t*)(c->ws + L.tkey);
  c->tb.count = (int32_t*)(c->ws + L.tcount);
  c->tb.start = (int32_t*)(c->ws + L.tstart);
  c->tb.cursor = (int32_t*)(c->ws + L.tcursor);
  c->tb.work = (int4*)(c->ws + L.twork);
  c->tb.nwork = (int32_t*)(c->ws + L.tnwork);
  c->sorted = (cfg->flags & PIC_FLAG_NO_SORT) == 0;
  {
    // a position update moves a particle by less than c dt; the window's slack
    // absorbs sort_every updates without any particle leaving it
    const double cells = cfg->c * cfg->dt / std::min(g.dx, g.dy);
    const int auto_every = std::max(1, (int)std::floor(c->tp.slack / std::max(cells, 1e-300)));
    c->sort_every = cfg->sort_interval > 0 ? cfg->sort_interval : std::min(auto_every, 64);
  }
  SchemeCoef& sc = c->sc;
  sc.scheme = cfg->scheme;
  sc.k = cfg->scheme == PIC_SCHEME_BDF ? cfg->bdf_order : 0;
  sc.dt = cfg->dt;
  sc.c = cfg->c;
  sc.eps0 = cfg->eps0;
  sc.mu0 = cfg->mu0;
  if (cfg->scheme == PIC_SCHEME_BDF) {
    // Sec. 3.2: C = a*a; alpha = a_0/(c dt) so that the solve divides by C_0
    bdf_coefficients(sc.k, sc.a);
    double C[13] = {0};
    for (int i = 0; i <= sc.k; ++i)
      for (int j = 0; j <= sc.k; ++j) C[i + j] += sc.a[i] * sc.a[j];
    for (int i = 0; i <= 2 * sc.k; ++i) sc.Cn[i] = C[i] / C[0];
    const double alpha = sc.a[0] / (cfg->c * cfg->dt);
    sc.inv_alpha2 = 1.0 / (alpha * alpha);
  } else if (cfg->scheme == PIC_SCHEME_CDF2) {
    sc.inv_alpha2 = 0.5 * cfg->c * cfg->c * cfg->dt * cfg->dt;  // alpha = sqrt(2)/(c dt), Sec. 3.1
  } else {
    // Qin-Zhang two-stage symplectic DIRK (the printed tableau in Sec. 5 is
    // garbled; this is the consistent second-order, |R(i theta)| = 1 scheme)
    sc.dirkA[0][0] = 0.25;
    sc.dirkA[0][1] = 0.0;
    sc.dirkA[1][0] = 0.5;
    sc.dirkA[1][1] = 0.25;
    sc.dirkB[0] = sc.dirkB[1] = 0.5;
    sc.dirkC[0] = 0.25;
    sc.dirkC[1] = 0.75;
  }
  // twiddles
  std::vector<double> tw(2 * (size_t)std::max(cfg->nx, cfg->ny));
  fft_make_twiddles(cfg->nx, tw.data());
  hipError_t e = hipMemcpy(c->twx(), tw.data(), (size_t)cfg->nx * 16, hipMemcpyHostToDevice);
  if (e == hipSuccess) {
    fft_make_twiddles(cfg->ny, tw.data());
    e = hipMemcpy(c->twy(), tw.data(), (size_t)cfg->ny * 16, hipMemcpyHostToDevice);
  }
  if (e != hipSuccess) {
    g_err = std::string("twiddle upload: ") + hipGetErrorString(e);
    delete c;
    return PIC_ERR_HIP;
  }
  if (c->sorted) {
    hipError_t ez = hipMemsetAsync(c->tb.count, 0, (size_t)c->tp.ntiles * 4, c->stream);
    if (ez != hipSuccess) {
      g_err = std::string("tile count clear: ") + hipGetErrorString(ez);
      delete c;
      return PIC_ERR_HIP;
    }
  }
  if (reset_fields(c) != PIC_OK) {
    g_err = c->err;
    delete c;
    return PIC_ERR_HIP;
  }
  *out = c;
  return PIC_OK;
}

void pic_destroy(pic_ctx_t ctx) { delete ctx; }

pic_status_t init_particles(pic_ctx_t c, int64_t n, const double* x, const double* y, const double* P) {
  if (!c) return PIC_ERR_INVALID_ARG;
  if (n < 0 || n > c->cfg.max_particles) return c->fail(PIC_ERR_INVALID_ARG, "n must be in [0, max_particles]");
  if (n > 0 && (!x || !y || !P)) return c->fail(PIC_ERR_INVALID_ARG, "x, y, P must be device pointers");
  c->vflip = 0;
  auto pa = c->parts();
  pic_status_t st = c->hip(launch_init_particles(c->cfg.particle_dtype, &pa, n, x, y, P, c->g, c->ph, c->stream),
                           "init launch");
  if (st) return st;
  st = reset_fields(c);
  if (st) return st;
  c->n = n;
  st = do_sort(c);
  if (st) return st;
  c->phase = READY;
  return PIC_OK;
}

pic_status_t deposit_current(pic_ctx_t c) {
  if (!c) return PIC_ERR_INVALID_ARG;
  if (c->phase != READY) return c->fail(PIC_ERR_STATE, "deposit_current needs phase READY");
  pic_status_t st = do_deposit(c);
  if (st) return st;
  c->phase = DEPOSITED;
  return PIC_OK;
}

pic_status_t field_solve(pic_ctx_t c) {
  if (!c) return PIC_ERR_INVALID_ARG;
  if (c->phase != DEPOSITED) return c->fail(PIC_ERR_STATE, "field_solve needs phase DEPOSITED");
  pic_status_t st = do_solve(c);
  if (st) return st;
  c->phase = SOLVED;
  return PIC_OK;
}

pic_status_t gather_push(pic_ctx_t c) {
  if (!c) return PIC_ERR_INVALID_ARG;
  if (c->phase != SOLVED) return c->fail(PIC_ERR_STATE, "gather_push needs phase SOLVED");
  pic_status_t st = do_gather_push(c, false);
  if (st) return st;
  c->phase = READY;
  return PIC_OK;
}

pic_status_t step(pic_ctx_t c, int32_t nsteps) {
  if (!c) return PIC_ERR_INVALID_ARG;
  if (nsteps < 0) return c->fail(PIC_ERR_INVALID_ARG, "nsteps must be >= 0");
  if (c->phase != READY) return c->fail(PIC_ERR_STATE, "step needs phase READY");
  if (nsteps == 0) return PIC_OK;
  const bool unfused = (c->cfg.flags & PIC_FLAG_UNFUSED_STEP) != 0;
  pic_status_t st = do_deposit(c);
  for (int s = 0; s < nsteps && !st; ++s) {
    st = do_solve(c);
    if (st) break;
    const bool last = s == nsteps - 1;
    if (last || unfused) {
      st = do_gather_push(c, false);
      if (!st && !last) st = do_deposit(c);
    } else {
      st = do_gather_push(c, true);
    }
  }
  // a failed launch leaves the state undefined; report it and require a reload
  c->phase = st ? EMPTY : READY;
  return st;
}

pic_status_t pic_get_particles(pic_ctx_t c, double* out) {
  if (!c) return PIC_ERR_INVALID_ARG;
  if (c->phase == EMPTY) return c->fail(PIC_ERR_STATE, "no particles loaded");
  if (c->n > 0 && !out) return c->fail(PIC_ERR_INVALID_ARG, "out is NULL");
  auto pa = c->parts();
  return c->hip(launch_get_particles(c->cfg.particle_dtype, &pa, c->n, out, c->stream), "get_particles");
}

pic_status_t pic_set_particles(pic_ctx_t c, const double* in) {
  if (!c) return PIC_ERR_INVALID_ARG;
  if (c->phase == EMPTY) return c->fail(PIC_ERR_STATE, "no particles loaded");
  if (c->n > 0 && !in) return c->fail(PIC_ERR_INVALID_ARG, "in is NULL");
  c->vflip = 0;
  auto pa = c->parts();
  pic_status_t st =
      c->hip(launch_set_particles(c->cfg.particle_dtype, &pa, c->n, in, c->g, c->stream), "set_particles");
  if (st) return st;
  st = do_sort(c);
  if (st) return st;
  c->phase = READY;
  return PIC_OK;
}

pic_status_t pic_get_field(pic_ctx_t c, int32_t which, double* dst) {
  if (!c) return PIC_ERR_INVALID_ARG;
  if (!dst) return c->fail(PIC_ERR_INVALID_ARG, "dst is NULL");
  const size_t plane = (size_t)c->cfg.nx * c->cfg.ny;
  if (which == PIC_FIELD_J) {
    if (c->phase != DEPOSITED) return c->fail(PIC_ERR_STATE, "J is valid in phase DEPOSITED");
    return c->hip(hipMemcpyAsync(dst, c->J(), 3 * plane * 8, hipMemcpyDeviceToDevice, c->stream), "copy J");
  }
  if (which == PIC_FIELD_MESH) {
    if (c->phase != SOLVED) return c->fail(PIC_ERR_STATE, "mesh fields are valid in phase SOLVED");
    return c->hip(hipMemcpyAsync(dst, c->F64(), 12 * plane * 8, hipMemcpyDeviceToDevice, c->stream),
                  "copy mesh fields");
  }
  return c->fail(PIC_ERR_INVALID_ARG, "unknown field id");
}


pic_status_t pic_get_history(pic_ctx_t c, double* dst) {
  if (!c) return PIC_ERR_INVALID_ARG;
  if (!dst) return c->fail(PIC_ERR_INVALID_ARG, "dst is NULL");
  return history_io(c, dst, true);
}

pic_status_t pic_set_history(pic_ctx_t c, const double* src) {
  if (!c) return PIC_ERR_INVALID_ARG;
  if (!src) return c->fail(PIC_ERR_INVALID_ARG, "src is NULL");
  if (c->phase == DEPOSITED || c->phase == SOLVED)
    return c->fail(PIC_ERR_STATE, "set_history needs phase READY or EMPTY");
  return history_io(c, const_cast<double*>(src), false);
}

pic_status_t pic_diagnostics(pic_ctx_t c, double* out) {
  if (!c) return PIC_ERR_INVALID_ARG;
  if (!out) return c->fail(PIC_ERR_INVALID_ARG, "out is NULL");
  // the newest level is the one written by the last update: slots of s = nupd
  HistSlots hs = c->slots(c->nupd);
  pic_status_t st = c->hip(launch_field_diag(c->H(), c->g, c->sc, hs, c->diag(), c->stream), "field diag");
  if (st) return st;
  auto pa = c->parts();
  st = c->hip(launch_particle_diag(c->cfg.particle_dtype, &pa, c->n, c->ph, c->diag() + 16, c->stream),
              "particle diag");
  if (st) return st;
  std::vector<double> h(16 + 512);
  st = c->hip(hipMemcpyAsync(h.data(), c->diag(), h.size() * 8, hipMemcpyDeviceToHost, c->stream), "diag copy");
  if (st) return st;
  st = c->hip(hipStreamSynchronize(c->stream), "diag sync");
  if (st) return st;
  for (int i = 0; i < 6; ++i) out[i] = h[i];
  double ke = 0, bad = 0;
  for (int b = 0; b < 256; ++b) {
    ke += h[16 + 2 * b];
    bad += h[16 + 2 * b + 1];
  }
  out[6] = ke;
  out[7] = bad;
  return bad > 0 ? c->fail(PIC_ERR_NONFINITE, "non-finite particle values") : PIC_OK;
}

pic_status_t pic_set_kernel_timing(pic_ctx_t c, int32_t enable) {
  if (!c) return PIC_ERR_INVALID_ARG;
  c->timing = enable != 0;
  return PIC_OK;
}

pic_status_t pic_kernel_timing(pic_ctx_t c, double* out) {
  if (!c) return PIC_ERR_INVALID_ARG;
  if (!out) return c->fail(PIC_ERR_INVALID_ARG, "out is NULL");
  pic_status_t st = c->hip(c->fold_timing(), "kernel timing");
  if (st) return st;
  for (int k = 0; k < PIC_KCLASS_COUNT; ++k) {
    out[2 * k] = c->t_ms[k];
    out[2 * k + 1] = c->t_n[k];
    c->t_ms[k] = c->t_n[k] = 0;
  }
  return PIC_OK;
}

}  // extern "C"
