// libpic C ABI: validation, workspace layout, phase state machine and launch
// sequencing of Algorithm 1 (arXiv 2410.18414, Sec. 4.2).
//
// A context holds one or more instances of the method (an ensemble); every
// hot-path kernel is launched once per phase over a flattened grid covering
// all instances, which advance in lockstep.  The plain API is a context of one
// instance.
#include <algorithm>
#include <array>
#include <atomic>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
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
inline int ceil_div(int64_t a, int64_t b) { return (int)((a + b - 1) / b); }
// one particle array of the given capacity, 256-byte aligned
inline size_t array_bytes(size_t cap, size_t es) { return align_up(cap * es); }

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

// the three centred-difference forms share the CDF-2 family's history and
// kernels; the form selects the wave update
int scheme_family(int scheme) {
  if (scheme == PIC_SCHEME_CDF2_SEMI || scheme == PIC_SCHEME_CDF2_EXPLICIT) return PIC_SCHEME_CDF2;
  return scheme == PIC_SCHEME_DIRK3 ? PIC_SCHEME_DIRK2 : scheme;  // every DIRK shares one layout
}
int cdf_form(int scheme) {
  return scheme == PIC_SCHEME_CDF2_SEMI ? 1 : (scheme == PIC_SCHEME_CDF2_EXPLICIT ? 2 : 0);
}

Hist plan_history(const pic_config_t& c) {
  Hist h;
  int b = 0;
  auto mk = [&](Ring& r, int size, int width) {
    r.base = b;
    r.size = size;
    r.width = width;
    b += size * width;
  };
  const int family = scheme_family(c.scheme);
  if (family == PIC_SCHEME_BDF) {
    const int k = c.bdf_order;
    mk(h.rho, k, 1);
    mk(h.phi, 2 * k, 1);
    mk(h.A, 2 * k, 3);
    h.nexport = k + 2 * k + 6 * k;
  } else if (family == PIC_SCHEME_CDF2) {
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
    mk(h.J, 2, 3);  // J^n read and J^{n+1} written by different blocks: two levels, the newest exported
    h.nexport = 17;
  }
  h.nslots = b;
  return h;
}

HistSlots slots_of(const Hist& r, int64_t s) {
  HistSlots h{};
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

bool validate(const pic_config_t* c, std::string& msg) {
  if (!c) { msg = "cfg is NULL"; return false; }
  if (c->abi_version != PIC_ABI_VERSION) { msg = "abi_version mismatch"; return false; }
  if (c->nx < 8 || c->ny < 8 || c->nx > 1024 || c->ny > 1024) {
    msg = "nx, ny must be in [8, 1024]";
    return false;
  }
  if (!(c->lx > 0) || !(c->ly > 0) || !std::isfinite(c->lx) || !std::isfinite(c->ly)) {
    msg = "lx, ly must be positive and finite";
    return false;
  }
  if (c->spline_degree < 1 || c->spline_degree > 5) { msg = "spline_degree must be 1..5"; return false; }
  if (c->scheme < PIC_SCHEME_BDF || c->scheme > PIC_SCHEME_DIRK3) { msg = "unknown scheme"; return false; }
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
  // the tiled passes wrap window offsets by one period on such grids
  if ((!pow2(c->nx) || !pow2(c->ny)) && (c->slack ? c->slack : 3) + 2 > std::min(c->nx, c->ny)) {
    msg = "slack must be at most min(nx, ny) - 2 on grids that are not powers of two";
    return false;
  }
  if (c->flags & ~(PIC_FLAG_NO_SORT | PIC_FLAG_UNFUSED_STEP | PIC_FLAG_NO_GRAPH | PIC_FLAG_ADJOINT |
                   PIC_FLAG_NAIVE_RHO | PIC_FLAG_JVSTAR | PIC_FLAG_DIRK_SUBSTEP | PIC_FLAG_DETERMINISTIC)) {
    msg = "unknown flag bits";
    return false;
  }
  for (int i = 0; i < 4; ++i)
    if (c->reserved[i]) { msg = "reserved fields must be zero"; return false; }
  return true;
}

// instances of one context must share the method (stepper, order, precision,
// spline, flags, c/eps0/mu0); grids, particle counts and time steps may differ
bool compatible(const pic_config_t& a, const pic_config_t& b, std::string& msg) {
  if (a.scheme != b.scheme || (a.scheme == PIC_SCHEME_BDF && a.bdf_order != b.bdf_order) ||
      a.particle_dtype != b.particle_dtype || a.spline_degree != b.spline_degree || a.flags != b.flags ||
      a.c != b.c || a.eps0 != b.eps0 || a.mu0 != b.mu0) {
    msg = "ensemble instances must share scheme, bdf_order, particle_dtype, spline_degree, flags, c, eps0, mu0";
    return false;
  }
  return true;
}

// Tile plan: tiles of 16x16 cells (smaller on small grids), a slack of three
// cells, chunks of at most 512 particles per workgroup, unless the config
// sets them.
TileP plan_tiles(const pic_config_t& c) {
  TileP t{};
  t.nx = c.nx;
  t.ny = c.ny;
  t.pow2 = pow2(c.nx) && pow2(c.ny) ? 1 : 0;
  // tile edge: a power of two not above either side (16 by default); a side
  // that is not a multiple of it ends in a partial tile
  int ts = 16;
  while (ts > std::min(c.nx, c.ny)) ts >>= 1;
  t.ts = c.tile_cells ? c.tile_cells : ts;
  t.ntx = (c.nx + t.ts - 1) / t.ts;
  t.nty = (c.ny + t.ts - 1) / t.ts;
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
  // default chunk: the largest of 512 .. 4096 particles that still leaves
  // at least 8192 chunks (32 per CU) at full capacity; bigger chunks amortise
  // the window load and flush once parallelism is plentiful
  int chunk = 512;
  while (chunk < 4096 && c.max_particles / (2 * chunk) >= 8192) chunk *= 2;
  t.chunk = c.chunk ? c.chunk : chunk;
  t.max_work = t.ntiles + ceil_div(c.max_particles, t.chunk);
  return t;
}

struct Layout {
  size_t set_bytes;  // one particle set: 11 arrays (cap x es) + ids
  size_t parts, J, T, RB, H, U, F64, F32, twx, twy, tcount, tstart, tcstart, ccount, ccursor, twork, tnwork, tdone,
      trank,
      LF, LS, LJ, LAM, LAM2, LIDS, LINV, LFLAG, total;
  size_t plane_c;    // complex entries per spectral plane
};

SchemeCoef make_scheme(const pic_config_t& c);

Layout plan_instance(const pic_config_t& c) {
  Layout L{};
  const size_t es = c.particle_dtype == PIC_F32 ? 4 : 8;
  const size_t cap = (size_t)c.max_particles;
  const size_t nxh = c.nx / 2 + 1;
  const size_t plane_r = (size_t)c.nx * c.ny;
  L.plane_c = nxh * c.ny;
  const Hist h = plan_history(c);
  const TileP tp = plan_tiles(c);
  size_t o = 0;
  auto take = [&](size_t bytes) {
    const size_t at = o;
    o = align_up(o + bytes);
    return at;
  };
  L.set_bytes = 11 * array_bytes(cap, es) + align_up(cap * 4);
  L.parts = take(2 * L.set_bytes);
  const bool naive = (c.flags & PIC_FLAG_NAIVE_RHO) != 0;
  const int njp = j_planes(make_scheme(c), naive ? 1 : 0);
  L.J = take(njp * plane_r * 8);
  L.T = take(njp * L.plane_c * 16);
  L.RB = naive ? take(plane_r * 8) : 0;
  L.H = take((size_t)h.nslots * L.plane_c * 16);
  L.U = take(8 * L.plane_c * 16);
  L.F64 = take(12 * plane_r * 8);
  L.F32 = c.particle_dtype == PIC_F32 ? take(12 * plane_r * 4) : 0;
  L.twx = take((size_t)c.nx * 16);
  L.twy = take((size_t)c.ny * 16);
  L.tcount = take((size_t)tp.ntiles * 4);
  L.tstart = take(((size_t)tp.ntiles + 1) * 4);
  L.tcstart = take((size_t)tp.ntiles * 4);
  const size_t ckeys = (size_t)tp.ntiles * tp.ts * tp.ts;  // cell keys (>= nx ny)
  L.ccount = take(ckeys * 4);
  L.ccursor = take(ckeys * 4);
  L.twork = take((size_t)tp.max_work * 16);
  L.tnwork = take(4);
  L.tdone = take(4);
  L.trank = take((size_t)cap * 4);
  if (c.flags & PIC_FLAG_ADJOINT) {
    L.LF = take(11 * plane_r * 8);
    L.LS = take(11 * L.plane_c * 16);
    L.LJ = take(3 * plane_r * 8);
    L.LAM = take(11 * cap * 8);
    L.LAM2 = take(11 * cap * 8);
    L.LIDS = take(cap * 4);
    L.LINV = take(cap * 4);
    L.LFLAG = take(4);
  }
  L.total = o;
  return L;
}

// context-level buffers ahead of the instances: descriptors and diagnostics
// diagnostics buffer: the field reduction's six values (16 slots), then 256
// block partials of the kinetic energy and the non-finite count
constexpr size_t kDiagDoubles = 16 + 2 * 256;
size_t head_bytes(int ninst) { return align_up(ninst * sizeof(InstDesc)) + align_up(kDiagDoubles * 8); }

size_t total_bytes(const pic_config_t* cfgs, int ninst) {
  size_t t = head_bytes(ninst);
  for (int i = 0; i < ninst; ++i) t += plan_instance(cfgs[i]).total;
  return t;
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

SchemeCoef make_scheme(const pic_config_t& c) {
  SchemeCoef sc{};
  sc.scheme = scheme_family(c.scheme);
  sc.form = cdf_form(c.scheme);
  sc.k = c.scheme == PIC_SCHEME_BDF ? c.bdf_order : 0;
  sc.dt = c.dt;
  sc.c = c.c;
  sc.eps0 = c.eps0;
  sc.mu0 = c.mu0;
  if (c.scheme == PIC_SCHEME_BDF) {
    // Sec. 3.2: C = a*a; alpha = a_0/(c dt) so that the solve divides by C_0
    bdf_coefficients(sc.k, sc.a);
    double C[13] = {0};
    for (int i = 0; i <= sc.k; ++i)
      for (int j = 0; j <= sc.k; ++j) C[i + j] += sc.a[i] * sc.a[j];
    for (int i = 0; i <= 2 * sc.k; ++i) sc.Cn[i] = C[i] / C[0];
    const double alpha = sc.a[0] / (c.c * c.dt);
    sc.inv_alpha2 = 1.0 / (alpha * alpha);
  } else if (sc.scheme == PIC_SCHEME_CDF2) {
    sc.inv_alpha2 = 0.5 * c.c * c.c * c.dt * c.dt;  // alpha = sqrt(2)/(c dt), Sec. 3.1 (explicit: c^2 dt^2 / 2)
  } else {
    // DIRK as a composition of implicit-midpoint substeps of lengths b_i dt:
    // a_ij = b_j (j < i), a_ii = b_i / 2, c_i = sum_j a_ij.  Two stages with
    // b = (1/2, 1/2) give the Qin-Zhang symplectic DIRK-2 (the printed
    // tableau in Sec. 5 is garbled; this is the consistent second-order,
    // |R(i theta)| = 1 scheme); three with the symmetric fourth-order weights
    // give DIRK-3.
    double b[3];
    if (c.scheme == PIC_SCHEME_DIRK3) {
      sc.stages = 3;
      b[0] = b[2] = 1.0 / (2.0 - std::cbrt(2.0));
      b[1] = 1.0 - 2.0 * b[0];
    } else {
      sc.stages = 2;
      b[0] = b[1] = 0.5;
    }
    sc.substep = (c.flags & PIC_FLAG_DIRK_SUBSTEP) ? 1 : 0;
    for (int i = 0; i < sc.stages; ++i) {
      sc.dirkB[i] = b[i];
      sc.dirkC[i] = 0.0;
      for (int j = 0; j < sc.stages; ++j) {
        sc.dirkA[i][j] = j < i ? b[j] : (j == i ? 0.5 * b[i] : 0.0);
        sc.dirkC[i] += sc.dirkA[i][j];
      }
    }
  }
  return sc;
}

struct Instance {
  pic_config_t cfg{};
  int every_worst = 1;  // sort interval if particles moved at c: slack / (c dt / min(dx, dy))
  int every = 1;        // this instance's sort interval (explicit, or from the loaded particles)
  Layout L{};
  size_t off = 0;  // byte offset of the instance region in the workspace
  InstDesc d{};    // host copy of the device descriptor
};

}  // namespace

// ---------------------------------------------------------------------------
// Scratch of pic_diagnostics_all: the per-instance reduction partials (the
// field reduction's six values, then 256 block partials of the kinetic energy
// and the non-finite count) of at most kDiagAllMax instances, in a
// file-scope device array.  Each GPU the library runs on holds its own copy
// until the process ends.  In host code the array's name is not a device
// address: host code uses only the address hipGetSymbolAddress returns for
// the current device, looked up once per device (scratch_on).
constexpr int kDiagAllMax = 64;
static __device__ __align__(256) double scratch[kDiagAllMax * kDiagDoubles];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double* g_scratch[kMaxDevices] = {};

// scratch's address on device dev (which must be current); nullptr on failure
double* scratch_on(int dev) {
  if (dev < 0 || dev >= kMaxDevices) return nullptr;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch[dev]) {
    void* ptr = nullptr;
    if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) return nullptr;
    g_scratch[dev] = static_cast<double*>(ptr);
  }
  return g_scratch[dev];
}

// out[i][0..5] = instance i's field values, out[i][6] = its kinetic energy,
// out[i][7] = its non-finite count: the block partials summed in block order,
// as pic_diagnostics sums them on the host
__global__ void k_diag_finalize(const double* __restrict__ part, int ninst, double* __restrict__ out) {
  const int i = blockIdx.x;
  if (i >= ninst || threadIdx.x != 0) return;
  const double* p = part + (size_t)i * kDiagDoubles;
  for (int k = 0; k < 6; ++k) out[i * PIC_DIAG_COUNT + k] = p[k];
  double ke = 0, bad = 0;
  for (int b = 0; b < 256; ++b) {
    ke += p[16 + 2 * b];
    bad += p[16 + 2 * b + 1];
  }
  out[i * PIC_DIAG_COUNT + 6] = ke;
  out[i * PIC_DIAG_COUNT + 7] = bad;
}

}  // namespace

// ---------------------------------------------------------------------------
// Saved states (pic_save_state / pic_load_state): a header (16 words: magic,
// configuration fingerprint, counters; then one particle count per instance),
// then per instance the current particle set (11 arrays and the original
// indices, n entries each), the tile metadata of the last sort (tile starts,
// each tile's first chunk, the chunk list and its length), the spectral
// history ring and, with the naive current, the background charge plane
// init_particles computed.  A save or a load is one kernel launch over a
// list of segments.
constexpr uint64_t kStateMagic = 0x70696373746174ull;  // "picstat"
constexpr int kStateHeaderWords = 16;

namespace {

struct HeaderWords {
  int64_t w[kStateHeaderWords];
};

__global__ void k_state_header(int64_t* h, HeaderWords hw, int count) {
  if ((int)threadIdx.x < count) h[threadIdx.x] = hw.w[threadIdx.x];
}

// copy every segment of the list: each workgroup copies one span of
// kCopySpan bytes of one segment (the segment found by a wave-uniform scan of
// the block prefix sums), every thread kCopyUnroll 16-byte vectors in flight;
// segments of 16 bytes or more start 16-byte aligned on both sides, a shorter
// tail goes in 4-byte words
constexpr int kCopyMax = 32;
constexpr int kCopyThreads = 256, kCopyUnroll = 4;
constexpr uint64_t kCopySpan = (uint64_t)kCopyThreads * kCopyUnroll * 16;
struct CopyList {
  int count;
  uint64_t first[kCopyMax + 1];  // prefix sums of the segments' spans (workgroups)
  const char* src[kCopyMax];
  char* dst[kCopyMax];
  uint64_t bytes[kCopyMax];
};

__global__ void __launch_bounds__(kCopyThreads) k_copy_list(CopyList L) {
  const uint64_t b = blockIdx.x;
  int sg = 0;
  while (sg + 1 < L.count && L.first[sg + 1] <= b) ++sg;
  const uint64_t base = (b - L.first[sg]) * kCopySpan;
  const uint64_t nbytes = L.bytes[sg];
  const gptr<const char> src = gp(L.src[sg]);
  const gptr<char> dst = gp(L.dst[sg]);
  i32x4 v[kCopyUnroll];
#pragma unroll
  for (int u = 0; u < kCopyUnroll; ++u) {
    const uint64_t off = base + (uint64_t)(u * kCopyThreads + threadIdx.x) * 16;
    if (off + 16 <= nbytes) v[u] = *reinterpret_cast<gptr<const i32x4>>(src + off);
  }
#pragma unroll
  for (int u = 0; u < kCopyUnroll; ++u) {
    const uint64_t off = base + (uint64_t)(u * kCopyThreads + threadIdx.x) * 16;
    if (off + 16 <= nbytes) {
      *reinterpret_cast<gptr<i32x4>>(dst + off) = v[u];
    } else if (off < nbytes) {
      for (uint64_t q = off; q < nbytes; q += 4)
        *reinterpret_cast<gptr<int32_t>>(dst + q) = *reinterpret_cast<gptr<const int32_t>>(src + q);
    }
  }
}

}  // namespace

static uint64_t new_order_tag() {
  static std::atomic<uint64_t> next{1};
  return next.fetch_add(1, std::memory_order_relaxed);
}

struct pic_ctx_s {
  std::vector<Instance> inst;
  int sel = 0;  // instance addressed by the per-instance entry points
  hipStream_t stream = nullptr;
  char* ws = nullptr;
  Hist hist{};
  InstDesc* d_desc = nullptr;
  double* d_diag = nullptr;
  double* d_scratch = nullptr;  // scratch's address on the context's device
  int nblk[BK_NKINDS] = {0};
  size_t lds_r2c = 0, lds_c2r = 0, lds_col = 0, lds_adj_col = 0, lds_tiled[3] = {0, 0, 0};
  int max_ny = 0;  // largest grid side in y over the instances (column kernel block size)
  int dtype = 0, degree = 3, scheme = 0;
  int geo = 0;  // compiled window geometry shared by every instance (0: none, runtime geometry)
  bool sorted = true;
  int sort_every = 4;
  int64_t nupd = 0;  // completed field updates (history head)
  int vflip = 0;     // 0: V0 holds v^n; 1: V1 holds v^n
  int cur = 0;       // current particle set
  int moves = 0;     // position updates since the last sort
  bool stepped = false;
  int64_t lam_n = -1;  // particle count of the held adjoint (-1: none)
  // the slot order of the current particle set: a process-wide serial taken
  // whenever the order is made (sort, initial load, import) and kept with
  // saved states, so that equal tags mean equal orders; lam_tag is the order
  // the held adjoint follows (0: unknown, checked on the device)
  uint64_t order_tag = new_order_tag();
  uint64_t lam_tag = 0;
  // the order and the tile metadata come from a sort of these particles (not
  // an initial load or an import): every particle is in its tile's chunks
  bool from_sort = false;
  // step_adjoint has run on the current phase-SOLVED state (a second call
  // would apply the same step's transpose again)
  bool adjoined = false;
  Phase phase = EMPTY;
  std::string err;

  // captured loop body: `gperiod` iterations (field solve + fused particle
  // pass, with the sorts they contain), valid from the state `gkey`
  bool use_graphs = true;
  hipStream_t cap_stream = nullptr;
  hipGraphExec_t gexec = nullptr;
  // second stream for the tile sort, which runs beside the field solve (the
  // sort reads and writes particle sets, the solve mesh arrays), with the
  // fork and join events
  hipStream_t side = nullptr;
  hipEvent_t ev_fork = nullptr, ev_join = nullptr;
  int gperiod = 0;
  int64_t gkey[4] = {-1, -1, -1, -1};
  int lr = 1;  // lcm of the history ring sizes

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
    if (gexec) (void)hipGraphExecDestroy(gexec);
    if (cap_stream) (void)hipStreamDestroy(cap_stream);
    if (side) (void)hipStreamDestroy(side);
    if (ev_fork) (void)hipEventDestroy(ev_fork);
    if (ev_join) (void)hipEventDestroy(ev_join);
    for (auto& e : ev) {
      if (e.a) (void)hipEventDestroy(e.a);
      if (e.b) (void)hipEventDestroy(e.b);
    }
  }
  int ninst() const { return (int)inst.size(); }
  Instance& I() { return inst[sel]; }
  StepArgs sargs(int stage = -1) const { return StepArgs{cur, vflip, stage}; }

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
    (void)hipEventRecord(p->a, stream);
    return p;
  }
  void end_timed(EvPair* p) {
    if (p) (void)hipEventRecord(p->b, stream);
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
  // upload the host descriptors (synchronises the stream; not on the step path)
  pic_status_t upload_desc() {
    std::vector<InstDesc> h(inst.size());
    for (size_t i = 0; i < inst.size(); ++i) h[i] = inst[i].d;
    hipError_t e = hipMemcpyAsync(d_desc, h.data(), h.size() * sizeof(InstDesc), hipMemcpyHostToDevice, stream);
    if (e == hipSuccess) e = hipStreamSynchronize(stream);
    return hip(e, "descriptor upload");
  }
};

namespace {

// counting sort of every instance's particles by tile into the other set
pic_status_t do_sort(pic_ctx_t c) {
  if (!c->sorted) return PIC_OK;
  auto* t = c->begin_timed(4);
  hipError_t e = launch_tile_sort(c->dtype, c->d_desc, c->ninst(), c->nblk[BK_COUNT], c->nblk[BK_TILES],
                                  c->nblk[BK_PART], c->cur, c->stream);
  c->end_timed(t);
  pic_status_t st = c->hip(e, "tile sort");
  if (st) return st;
  c->cur ^= 1;
  c->moves = 0;
  c->order_tag = new_order_tag();
  c->from_sort = true;
  return PIC_OK;
}

// sort first when the next position update could carry a particle past the slack
pic_status_t maybe_sort(pic_ctx_t c) {
  if (c->sorted && c->moves >= c->sort_every) return do_sort(c);
  return PIC_OK;
}

// mode: 0 deposit, 1 gather + push, 2 fused.  may_sort false: no sort even
// when one is due (the particles keep their order; a particle that drifted
// past its window takes the global path)
pic_status_t particle_pass(pic_ctx_t c, int mode, bool may_sort = true) {
  // the phases start with a deposit, so a sort due after loading happens there
  if (mode != 1 && may_sort) {
    pic_status_t st = maybe_sort(c);
    if (st) return st;
  }
  static const int cls[3] = {0, 2, 3};
  auto* t = c->begin_timed(cls[mode]);
  // sub-stepped DIRK currents: one deposit pass per stage (the last one also
  // writes x^{n+1})
  const SchemeCoef& sc = c->inst[0].d.sc;
  const int nst = mode == 0 && sc.substep ? sc.stages : 0;
  hipError_t e = hipSuccess;
  for (int k = nst ? 0 : -1; k < nst && e == hipSuccess; ++k)
    e = c->sorted ? launch_tiled(c->dtype, mode, c->degree, c->geo, c->d_desc, c->ninst(), c->nblk[BK_WORK],
                                 c->lds_tiled[mode], c->sargs(k), c->stream)
                  : launch_untiled(c->dtype, mode, c->degree, c->d_desc, c->ninst(), c->nblk[BK_PART], c->sargs(k),
                                   c->stream);
  c->end_timed(t);
  pic_status_t st = c->hip(e, "particle pass");
  if (st) return st;
  if (mode != 1) c->moves += 1;
  if (mode != 0) c->vflip ^= 1;  // v^{n+1} was written over v^{n-1}
  c->stepped = true;
  return PIC_OK;
}

pic_status_t do_solve(pic_ctx_t c) {
  auto* t = c->begin_timed(1);
  const int ni = c->ninst();
  pic_status_t st = c->hip(launch_rows_r2c(c->d_desc, ni, c->nblk[BK_R2C], c->lds_r2c, c->stream), "rows_r2c");
  if (!st)
    st = c->hip(launch_columns(c->scheme, c->inst[0].cfg.bdf_order, c->d_desc, ni, c->nblk[BK_COL], c->lds_col,
                               slots_of(c->hist, c->nupd), c->max_ny, c->stream),
                "columns");
  if (!st) st = c->hip(launch_rows_c2r(c->d_desc, ni, c->nblk[BK_C2R], c->lds_c2r, c->stream), "rows_c2r");
  c->end_timed(t);
  if (st) return st;
  c->nupd += 1;
  c->stepped = true;
  c->adjoined = false;
  return PIC_OK;
}

pic_status_t reset_fields(pic_ctx_t c, Instance& in) {
  const InstDesc& d = in.d;
  pic_status_t st = c->hip(launch_fill_f64((double*)d.H, (size_t)c->hist.nslots * in.L.plane_c * 2, 0.0, c->stream),
                           "history fill");
  if (st) return st;
  // every J plane but the naive mode's rho plane (set to the ion background by init_particles)
  st = c->hip(launch_fill_f64(d.J, (size_t)j_planes(d.sc, 0) * in.cfg.nx * in.cfg.ny, 0.0, c->stream), "J fill");
  if (st || !d.LF) return st;
  return c->hip(launch_fill_f64(d.LF, (size_t)11 * in.cfg.nx * in.cfg.ny, 0.0, c->stream), "adjoint fill");
}

struct PartsAny {
  union {
    Parts<float> f;
    Parts<double> d;
  };
};
PartsAny parts_of(pic_ctx_t c, const InstDesc& d, int set) {
  PartsAny a;
  if (c->dtype == PIC_F32) a.f = make_parts<float>(d, set, c->vflip);
  else a.d = make_parts<double>(d, set, c->vflip);
  return a;
}

pic_status_t create(const pic_config_t* cfgs, int ninst, void* workspace, size_t ws_bytes, void* hip_stream,
                    pic_ctx_t* out) {
  std::string m;
  if (!out) {
    g_err = "out is NULL";
    return PIC_ERR_INVALID_ARG;
  }
  *out = nullptr;
  if (!cfgs || ninst < 1 || ninst > 4096) {
    g_err = "need 1..4096 configs";
    return PIC_ERR_INVALID_ARG;
  }
  for (int i = 0; i < ninst; ++i) {
    if (!validate(&cfgs[i], m) || !compatible(cfgs[0], cfgs[i], m)) {
      g_err = ninst > 1 ? "instance " + std::to_string(i) + ": " + m : m;
      return PIC_ERR_INVALID_ARG;
    }
  }
  if ((cfgs[0].flags & PIC_FLAG_DETERMINISTIC) &&
      (cfgs[0].flags & (PIC_FLAG_NO_SORT | PIC_FLAG_NAIVE_RHO | PIC_FLAG_ADJOINT))) {
    g_err = "the deterministic deposit needs the sorted passes (not with NO_SORT, NAIVE_RHO or ADJOINT)";
    return PIC_ERR_UNSUPPORTED;
  }
  if (cfgs[0].flags & PIC_FLAG_DIRK_SUBSTEP) {
    if (scheme_family(cfgs[0].scheme) != PIC_SCHEME_DIRK2) {
      g_err = "sub-stepped stage currents need a DIRK scheme";
      return PIC_ERR_UNSUPPORTED;
    }
    if (cfgs[0].flags & (PIC_FLAG_NAIVE_RHO | PIC_FLAG_ADJOINT)) {
      g_err = "sub-stepped stage currents are not available with the naive deposit or the adjoint";
      return PIC_ERR_UNSUPPORTED;
    }
  }
  if (cfgs[0].flags & PIC_FLAG_ADJOINT) {
    for (int i = 0; i < ninst; ++i)
      if (!pow2(cfgs[i].nx) || !pow2(cfgs[i].ny)) {
        g_err = "the adjoint needs power-of-two grid sides";
        return PIC_ERR_UNSUPPORTED;
      }
  }
  if ((cfgs[0].flags & PIC_FLAG_JVSTAR) && (cfgs[0].flags & PIC_FLAG_ADJOINT)) {
    g_err = "the adjoint is not available with v* in the current";
    return PIC_ERR_UNSUPPORTED;
  }
  if (cfgs[0].flags & PIC_FLAG_NAIVE_RHO) {
    if (scheme_family(cfgs[0].scheme) == PIC_SCHEME_CDF2) {
      g_err = "the naive charge deposit needs BDF-k or DIRK-2 (CDF-2 needs rho at half levels)";
      return PIC_ERR_UNSUPPORTED;
    }
    if (cfgs[0].flags & PIC_FLAG_ADJOINT) {
      g_err = "the adjoint is not available with the naive charge deposit";
      return PIC_ERR_UNSUPPORTED;
    }
  }
  const size_t need = total_bytes(cfgs, ninst);
  if (!workspace || ((uintptr_t)workspace & (kAlign - 1))) {
    g_err = "workspace must be a 256-byte aligned device pointer";
    return PIC_ERR_WORKSPACE;
  }
  if (ws_bytes < need) {
    g_err = "workspace too small: need " + std::to_string(need) + " bytes";
    return PIC_ERR_WORKSPACE;
  }
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) {
    g_err = "hipGetDevice failed";
    return PIC_ERR_HIP;
  }
  int max_lds = 0;
  if (hipDeviceGetAttribute(&max_lds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess) {
    g_err = "hipDeviceGetAttribute (LDS per block) failed";
    return PIC_ERR_HIP;
  }
  double* scr = scratch_on(dev);
  if (!scr) {
    g_err = "hipGetSymbolAddress of the diagnostics scratch failed";
    return PIC_ERR_HIP;
  }
  auto* c = new pic_ctx_s();
  c->d_scratch = scr;
  c->stream = (hipStream_t)hip_stream;
  c->ws = (char*)workspace;
  c->hist = plan_history(cfgs[0]);
  {
    auto lcm = [](int a, int b) {
      int x = a, y = b;
      while (y) {
        const int t = x % y;
        x = y;
        y = t;
      }
      return a / x * b;
    };
    const Hist& h = c->hist;
    c->lr = lcm(lcm(lcm(h.rho.size, h.phi.size), lcm(h.A.size, h.J.size)), 1);
  }
  c->use_graphs = (cfgs[0].flags & PIC_FLAG_NO_GRAPH) == 0;
  c->dtype = cfgs[0].particle_dtype;
  c->degree = cfgs[0].spline_degree;
  c->scheme = scheme_family(cfgs[0].scheme);
  c->sorted = (cfgs[0].flags & PIC_FLAG_NO_SORT) == 0;
  c->d_desc = (InstDesc*)c->ws;
  c->d_diag = (double*)(c->ws + align_up(ninst * sizeof(InstDesc)));
  c->inst.resize(ninst);
  size_t off = head_bytes(ninst);
  int every = 64;
  std::vector<double> tw;
  hipError_t e = hipSuccess;
  for (int i = 0; i < ninst && e == hipSuccess; ++i) {
    Instance& in = c->inst[i];
    const pic_config_t& cf = cfgs[i];
    in.cfg = cf;
    in.L = plan_instance(cf);
    in.off = off;
    off += in.L.total;
    char* b = c->ws + in.off;
    InstDesc& d = in.d;
    GridP& g = d.g;
    g.nx = cf.nx;
    g.ny = cf.ny;
    g.nxh = cf.nx / 2 + 1;
    g.lx = cf.lx;
    g.ly = cf.ly;
    g.dx = cf.lx / cf.nx;
    g.dy = cf.ly / cf.ny;
    g.inv_dx = 1.0 / g.dx;
    g.inv_dy = 1.0 / g.dy;
    g.inv_area = 1.0 / (g.dx * g.dy);
    d.ph = PhysP{cf.dt, cf.q, cf.m, cf.c};
    d.tp = plan_tiles(cf);
    d.sc = make_scheme(cf);
    const size_t es = cf.particle_dtype == PIC_F32 ? 4 : 8;
    const size_t cb = array_bytes((size_t)cf.max_particles, es);
    for (int s = 0; s < 2; ++s) {
      char* sb = b + in.L.parts + s * in.L.set_bytes;
      for (int k = 0; k < 11; ++k) d.set[s][k] = sb + k * cb;
      d.ids[s] = (int32_t*)(sb + 11 * cb);
    }
    d.J = (double*)(b + in.L.J);
    d.T = (double2*)(b + in.L.T);
    d.H = (double2*)(b + in.L.H);
    d.U = (double2*)(b + in.L.U);
    d.F64 = (double*)(b + in.L.F64);
    d.F32 = cf.particle_dtype == PIC_F32 ? (float*)(b + in.L.F32) : nullptr;
    d.twx = (const double2*)(b + in.L.twx);
    d.twy = (const double2*)(b + in.L.twy);
    d.tb.count = (int32_t*)(b + in.L.tcount);
    d.tb.start = (int32_t*)(b + in.L.tstart);
    d.tb.ccount = (int32_t*)(b + in.L.ccount);
    d.tb.ccursor = (int32_t*)(b + in.L.ccursor);
    d.tb.work = (int4*)(b + in.L.twork);
    d.tb.cstart = (int32_t*)(b + in.L.tcstart);
    d.tb.nwork = (int32_t*)(b + in.L.tnwork);
    d.tb.done = (int32_t*)(b + in.L.tdone);
    d.tb.rank = (int32_t*)(b + in.L.trank);
    const bool adj = (cf.flags & PIC_FLAG_ADJOINT) != 0;
    d.LF = adj ? (double*)(b + in.L.LF) : nullptr;
    d.LS = adj ? (double2*)(b + in.L.LS) : nullptr;
    d.LJ = adj ? (double*)(b + in.L.LJ) : nullptr;
    d.LAM = adj ? (double*)(b + in.L.LAM) : nullptr;
    d.LAM2 = adj ? (double*)(b + in.L.LAM2) : nullptr;
    d.LIDS = adj ? (int32_t*)(b + in.L.LIDS) : nullptr;
    d.LINV = adj ? (int32_t*)(b + in.L.LINV) : nullptr;
    d.LFLAG = adj ? (int32_t*)(b + in.L.LFLAG) : nullptr;
    d.naive = (cf.flags & PIC_FLAG_NAIVE_RHO) ? 1 : 0;
    d.jvstar = (cf.flags & PIC_FLAG_JVSTAR) ? 1 : 0;
    {
      // fixed-point deposit exponent (float32 particles): the largest single
      // contribution B = |q| c max(w) / (dx dy), max(w) = M_deg(0)^2, |v| < c
      // (3c for v*; the naive charge deposit's |q| max(w) / (dx dy) when that
      // is larger); B = m 2^p with m in [0.5, 1) gives B 2^(30 - p) < 2^30
      static const double m0[6] = {0.0, 1.0, 0.75, 2.0 / 3.0, 115.0 / 192.0, 0.55};
      const double vb = std::max(cf.c * ((cf.flags & PIC_FLAG_JVSTAR) ? 3.0 : 1.0),
                                 (cf.flags & PIC_FLAG_NAIVE_RHO) ? 1.0 : 0.0);
      const double B = std::fabs(cf.q) * vb * g.inv_area * m0[cf.spline_degree] * m0[cf.spline_degree];
      int p = 0;
      const bool ok = B > 0 && std::isfinite(B);
      if (ok) std::frexp(B, &p);
      d.qe0 = ok ? 30 - p : 0;
      // deterministic deposit: one scale for every contribution of the
      // instance.  Float32: the window scale of a full chunk (a chunk's sum
      // below 2^30, so int64 sums of every chunk cannot overflow).  Float64:
      // capacity x B 2^e < 2^62 bounds every int64 sum, window or global.
      d.det = (cf.flags & PIC_FLAG_DETERMINISTIC) ? 1 : 0;
      int cl2_chunk = 0, cl2_cap = 0;
      while ((1 << cl2_chunk) < d.tp.chunk) ++cl2_chunk;
      while (((int64_t)1 << cl2_cap) < cf.max_particles) ++cl2_cap;
      int e = cf.particle_dtype == PIC_F32 ? d.qe0 - std::max(cl2_chunk, 9) : (ok ? 62 - p - cl2_cap : 0);
      e = cf.particle_dtype == PIC_F32 ? std::max(-100, std::min(100, e)) : std::max(-1000, std::min(1000, e));
      d.qe_det = e;
      d.det_scale = std::ldexp(1.0, e);
      d.det_unscale = std::ldexp(1.0, -e);
    }
    d.RB = d.naive ? (double*)(b + in.L.RB) : nullptr;
    d.n = 0;
    d.R_r2c = rows_r2c_R(cf.nx, cf.ny);
    d.R_c2r = rows_c2r_R(cf.nx, cf.ny);
    d.nb_col = columns_nb(cf.ny);
    // flattened block ranges
    const int nb[BK_NKINDS] = {ceil_div(cf.ny, d.R_r2c) * j_planes(d.sc, d.naive),
                               (cf.nx / 2 + 1) * columns_parts(scheme_family(cf.scheme)),
                               ceil_div(cf.ny, d.R_c2r) * 6, d.tp.max_work,
                               ceil_div(cf.max_particles, 256), ceil_div(cf.max_particles, 1024),
                               ceil_div(d.tp.ntiles, 4)};
    for (int k = 0; k < BK_NKINDS; ++k) {
      d.blk[k] = c->nblk[k];
      c->nblk[k] += nb[k];
    }
    c->lds_r2c = std::max(c->lds_r2c, rows_r2c_lds_bytes(cf.nx, cf.ny));
    c->lds_c2r = std::max(c->lds_c2r, rows_c2r_lds_bytes(cf.nx, cf.ny));
    c->lds_col = std::max(c->lds_col, columns_split_lds_bytes(cf.ny, d.sc.substep ? d.sc.stages : 0));
    c->max_ny = std::max(c->max_ny, cf.ny);
    if (cf.flags & PIC_FLAG_ADJOINT) c->lds_adj_col = std::max(c->lds_adj_col, adj_columns_lds_bytes(cf.ny));
    for (int mode = 0; mode < 3; ++mode)
      c->lds_tiled[mode] = std::max(c->lds_tiled[mode], tiled_lds_bytes(cf.particle_dtype, mode, d.tp, d.naive != 0));
    // a position update moves a particle by less than c dt; the window's slack
    // absorbs sort_every updates without any particle leaving it
    const double cells = cf.c * cf.dt / std::min(g.dx, g.dy);
    const int auto_every = std::max(1, (int)std::floor(d.tp.slack / std::max(cells, 1e-300)));
    in.every_worst = std::min(auto_every, 64);
    in.every = cf.sort_interval > 0 ? cf.sort_interval : in.every_worst;
    every = std::min(every, in.every);
    // twiddles
    tw.assign(2 * (size_t)std::max(cf.nx, cf.ny), 0.0);
    fft_make_twiddles(cf.nx, tw.data());
    e = hipMemcpy((void*)d.twx, tw.data(), (size_t)cf.nx * 16, hipMemcpyHostToDevice);
    if (e == hipSuccess) {
      fft_make_twiddles(cf.ny, tw.data());
      e = hipMemcpy((void*)d.twy, tw.data(), (size_t)cf.ny * 16, hipMemcpyHostToDevice);
    }
    if (e == hipSuccess) e = hipMemset(d.tb.count, 0, (size_t)d.tp.ntiles * 4);
    if (e == hipSuccess) e = hipMemset(d.tb.ccount, 0, (size_t)d.tp.ntiles * d.tp.ts * d.tp.ts * 4);
    if (e == hipSuccess) e = hipMemset(d.tb.done, 0, 4);
  }
  c->sort_every = every;
  c->geo = tiled_geometry(c->inst[0].d.tp);
  for (int i = 1; i < ninst; ++i)
    if (tiled_geometry(c->inst[i].d.tp) != c->geo) c->geo = 0;
  if (e != hipSuccess) {
    g_err = std::string("context setup: ") + hipGetErrorString(e);
    delete c;
    return PIC_ERR_HIP;
  }
  size_t lds_need = std::max({c->lds_col, c->lds_adj_col, c->lds_r2c, c->lds_c2r});
  if (c->sorted) lds_need = std::max({lds_need, c->lds_tiled[0], c->lds_tiled[1], c->lds_tiled[2]});
  if (lds_need > (size_t)max_lds) {
    g_err = "grid or tile too large for this device's LDS";
    delete c;
    return PIC_ERR_UNSUPPORTED;
  }
  pic_status_t st = c->upload_desc();
  for (int i = 0; i < ninst && !st; ++i) st = reset_fields(c, c->inst[i]);
  if (!st) st = c->hip(hipStreamCreateWithFlags(&c->side, hipStreamNonBlocking), "sort stream");
  if (!st) st = c->hip(hipEventCreateWithFlags(&c->ev_fork, hipEventDisableTiming), "sort fork event");
  if (!st) st = c->hip(hipEventCreateWithFlags(&c->ev_join, hipEventDisableTiming), "sort join event");
  if (st) {
    g_err = c->err;
    delete c;
    return st;
  }
  c->moves = c->sort_every;  // sort before the first particle pass
  *out = c;
  return PIC_OK;
}

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
  if (c->scheme == PIC_SCHEME_DIRK2) ring(h.vphi, 1);
  ring(h.A, h.A.size);
  if (c->scheme == PIC_SCHEME_DIRK2) ring(h.vA, 1);
  if (c->scheme != PIC_SCHEME_BDF) ring(h.J, c->scheme == PIC_SCHEME_DIRK2 ? 1 : h.J.size);
  return v;
}

pic_status_t history_io(pic_ctx_t c, double* ext, bool to_external) {
  const std::vector<int> slots = export_slots(c);
  Instance& in = c->I();
  const size_t plane = in.L.plane_c;
  for (size_t f = 0; f < slots.size(); ++f) {
    double2* in_slot = in.d.H + (size_t)slots[f] * plane;
    double2* ext_f = (double2*)ext + f * plane;
    hipError_t e = to_external ? launch_hist_transpose(in_slot, ext_f, 1, in.d.g, true, c->stream)
                               : launch_hist_transpose(ext_f, in_slot, 1, in.d.g, false, c->stream);
    if (e != hipSuccess) return c->hip(e, "history transpose");
  }
  return PIC_OK;
}

// one loop iteration of a multi-step call: field solve, then the gather/push
// of this step fused with the next step's position update and deposit.  A
// sort due before the fused pass runs on the second stream beside the solve
// (direct launches and captured graphs alike; not while kernel timing is on,
// so that the timed classes do not overlap).
pic_status_t loop_body(pic_ctx_t c, bool unfused) {
  if (!unfused && !c->timing && c->sorted && c->moves >= c->sort_every) {
    hipStream_t main = c->stream;
    pic_status_t st = c->hip(hipEventRecord(c->ev_fork, main), "sort fork");
    if (!st) st = c->hip(hipStreamWaitEvent(c->side, c->ev_fork, 0), "sort fork wait");
    if (!st) {
      c->stream = c->side;
      st = do_sort(c);
      c->stream = main;
    }
    if (!st) st = c->hip(hipEventRecord(c->ev_join, c->side), "sort join");
    if (!st) st = do_solve(c);
    if (!st) st = c->hip(hipStreamWaitEvent(main, c->ev_join, 0), "sort join wait");
    if (!st) st = particle_pass(c, 2);
    return st;
  }
  pic_status_t st = do_solve(c);
  if (st) return st;
  if (unfused) {
    st = particle_pass(c, 1);
    if (!st) st = particle_pass(c, 0);
    return st;
  }
  return particle_pass(c, 2);
}

// steps per replayed graph: the launch state (history ring slots, velocity
// and particle-set flips, position updates since the sort) repeats after
// lcm(ring sizes, 2 sort intervals); 0 when step() does not use graphs
int graph_period(pic_ctx_t c) {
  int period = 2 * c->sort_every;
  while (period % c->lr) period += 2 * c->sort_every;
  return period <= 512 ? period : 0;
}

void state_key(pic_ctx_t c, int64_t* k) {
  k[0] = c->nupd % c->lr;
  k[1] = c->vflip;
  k[2] = c->cur;
  k[3] = c->moves;
}

// capture `period` loop iterations into a graph and launch it once (the
// capture itself advances the host-side state by `period` iterations)
pic_status_t capture_and_launch(pic_ctx_t c, bool unfused, int period) {
  if (c->gexec) {
    (void)hipGraphExecDestroy(c->gexec);
    c->gexec = nullptr;
  }
  if (!c->cap_stream) {
    pic_status_t st = c->hip(hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking), "capture stream");
    if (st) return st;
  }
  int64_t k0[4], k1[4];
  state_key(c, k0);
  hipStream_t user = c->stream;
  // the capture stream starts after the work already on the user stream
  hipEvent_t ev;
  pic_status_t st = c->hip(hipEventCreateWithFlags(&ev, hipEventDisableTiming), "capture event");
  if (st) return st;
  st = c->hip(hipEventRecord(ev, user), "capture event record");
  if (!st) st = c->hip(hipStreamWaitEvent(c->cap_stream, ev, 0), "capture wait");
  (void)hipEventDestroy(ev);
  if (st) return st;
  st = c->hip(hipStreamBeginCapture(c->cap_stream, hipStreamCaptureModeRelaxed), "begin capture");
  if (st) return st;
  c->stream = c->cap_stream;
  for (int i = 0; i < period && !st; ++i) st = loop_body(c, unfused);
  c->stream = user;
  hipGraph_t graph = nullptr;
  pic_status_t st2 = c->hip(hipStreamEndCapture(c->cap_stream, &graph), "end capture");
  if (st || st2) {
    if (graph) (void)hipGraphDestroy(graph);
    return st ? st : st2;
  }
  st = c->hip(hipGraphInstantiate(&c->gexec, graph, nullptr, nullptr, 0), "graph instantiate");
  (void)hipGraphDestroy(graph);
  if (st) return st;
  state_key(c, k1);
  c->gperiod = period;
  for (int i = 0; i < 4; ++i) c->gkey[i] = k0[i];
  if (k0[0] != k1[0] || k0[1] != k1[1] || k0[2] != k1[2] || k0[3] != k1[3]) c->gperiod = 0;  // not periodic
  return c->hip(hipGraphLaunch(c->gexec, user), "graph launch");
}

pic_status_t run_steps(pic_ctx_t c, int32_t nsteps) {
  if (!c) return PIC_ERR_INVALID_ARG;
  if (nsteps < 0) return c->fail(PIC_ERR_INVALID_ARG, "nsteps must be >= 0");
  if (c->phase != READY) return c->fail(PIC_ERR_STATE, "step needs phase READY");
  if (nsteps == 0) return PIC_OK;
  // sub-stepped DIRK currents need their own deposit passes after the push
  const bool unfused = (c->inst[0].cfg.flags & PIC_FLAG_UNFUSED_STEP) != 0 || c->inst[0].d.sc.substep;
  pic_status_t st = particle_pass(c, 0);
  int iters = nsteps - 1;
  // the host-side launch state repeats after lcm(ring sizes, 2 sort intervals)
  // iterations: replay one captured period while the state matches it
  const int period = graph_period(c);
  const bool graphs = c->use_graphs && !c->timing && c->sorted && period > 0;
  while (!st && graphs && iters >= period) {
    int64_t k[4];
    state_key(c, k);
    const bool have = c->gexec && c->gperiod == period;
    const bool match = have && k[0] == c->gkey[0] && k[1] == c->gkey[1] && k[2] == c->gkey[2] &&
                       k[3] == c->gkey[3];
    if (match) {
      st = c->hip(hipGraphLaunch(c->gexec, c->stream), "graph launch");
      c->nupd += period;  // vflip, cur and moves return to their values
      c->stepped = true;
      iters -= period;
    } else if (have) {
      // the captured period starts at another point of the cycle: step
      // eagerly up to it (fewer than `period` iterations) and keep the graph
      st = loop_body(c, unfused);
      iters -= 1;
    } else {
      st = capture_and_launch(c, unfused, period);
      iters -= period;
    }
  }
  for (int s = 0; s < iters && !st; ++s) st = loop_body(c, unfused);
  if (!st) st = do_solve(c);
  if (!st) st = particle_pass(c, 1);
  // a failed launch leaves the state undefined; report it and require a reload
  c->phase = st ? EMPTY : READY;
  return st;
}

}  // namespace

extern "C" {

size_t pic_workspace_bytes(const pic_config_t* cfg) {
  std::string m;
  if (!validate(cfg, m)) {
    g_err = m;
    return 0;
  }
  return total_bytes(cfg, 1);
}

size_t pic_batch_workspace_bytes(const pic_config_t* cfgs, int32_t ninst) {
  std::string m;
  if (!cfgs || ninst < 1 || ninst > 4096) {
    g_err = "need 1..4096 configs";
    return 0;
  }
  for (int i = 0; i < ninst; ++i)
    if (!validate(&cfgs[i], m) || !compatible(cfgs[0], cfgs[i], m)) {
      g_err = "instance " + std::to_string(i) + ": " + m;
      return 0;
    }
  return total_bytes(cfgs, ninst);
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
  if (!cfg) {
    g_err = "cfg is NULL";
    if (out) *out = nullptr;
    return PIC_ERR_INVALID_ARG;
  }
  return create(cfg, 1, workspace, ws_bytes, hip_stream, out);
}

pic_status_t pic_batch_create(const pic_config_t* cfgs, int32_t ninst, void* workspace, size_t ws_bytes,
                              void* hip_stream, pic_ctx_t* out) {
  return create(cfgs, ninst, workspace, ws_bytes, hip_stream, out);
}

void pic_destroy(pic_ctx_t ctx) { delete ctx; }

int32_t pic_instance_count(pic_ctx_t c) { return c ? c->ninst() : 0; }

pic_status_t pic_select_instance(pic_ctx_t c, int32_t i) {
  if (!c) return PIC_ERR_INVALID_ARG;
  if (i < 0 || i >= c->ninst()) return c->fail(PIC_ERR_INVALID_ARG, "instance index out of range");
  c->sel = i;
  return PIC_OK;
}

pic_status_t init_particles(pic_ctx_t c, int64_t n, const double* x, const double* y, const double* P) {
  if (!c) return PIC_ERR_INVALID_ARG;
  Instance& in = c->I();
  if (n < 0 || n > in.cfg.max_particles) return c->fail(PIC_ERR_INVALID_ARG, "n must be in [0, max_particles]");
  if (n > 0 && (!x || !y || !P)) return c->fail(PIC_ERR_INVALID_ARG, "x, y, P must be device pointers");
  if (c->ninst() > 1 && c->stepped)
    return c->fail(PIC_ERR_STATE, "ensemble instances are loaded before the first step");
  if (c->ninst() == 1) {  // a fresh start: counters and sets back to their initial state
    c->vflip = 0;
    c->cur = 0;
    c->nupd = 0;
    c->stepped = false;
  }
  auto pa = parts_of(c, in.d, c->cur);
  c->order_tag = new_order_tag();
  c->from_sort = false;
  pic_status_t st =
      c->hip(launch_init_particles(c->dtype, &pa, n, x, y, P, in.d.g, in.d.ph, c->stream), "init launch");
  if (st) return st;
  st = reset_fields(c, in);
  if (st) return st;
  if (in.d.naive) {
    // naive charge deposit: immobile ions = minus the electron charge at x^0,
    // which is also where the deposited rho plane of J starts
    const size_t plane = (size_t)in.cfg.nx * in.cfg.ny;
    st = c->hip(launch_fill_f64(in.d.RB, plane, 0.0, c->stream), "ion background fill");
    if (!st)
      st = c->hip(launch_charge(c->dtype, c->degree, &pa, n, in.d.g, -in.d.ph.q * in.d.g.inv_area, in.d.RB,
                                c->stream),
                  "ion background");
    if (!st)
      st = c->hip(hipMemcpyAsync(in.d.J + 3 * plane, in.d.RB, plane * sizeof(double), hipMemcpyDeviceToDevice,
                                 c->stream),
                  "rho plane start");
    if (st) return st;
  }
  in.d.n = n;
  st = c->upload_desc();
  if (st) return st;
  if (in.cfg.sort_interval == 0 && n > 0) {
    // sort interval from the loaded particles: a position update moves a
    // particle by at most max(|v_x|, |v_y|) dt in x and y, so the window's
    // slack lasts slack / (that / min(dx, dy)) updates; kept between the
    // speed-of-light interval and three times it (longer intervals let
    // particles that speed up escape their windows, and let the cell order
    // inside a tile decay, enough to cost more in the fused pass than they
    // save in sorts).  A particle that outruns it takes
    // the global path until the next sort, so results never depend on it.
    uint32_t* d_vmax = reinterpret_cast<uint32_t*>(c->d_diag);
    uint32_t h_vmax = 0;
    st = c->hip(hipMemsetAsync(d_vmax, 0, sizeof(uint32_t), c->stream), "speed reset");
    if (!st) st = c->hip(launch_max_inplane(c->dtype, &pa, n, d_vmax, c->stream), "speed launch");
    if (!st) st = c->hip(hipMemcpyAsync(&h_vmax, d_vmax, sizeof(uint32_t), hipMemcpyDeviceToHost, c->stream), "speed copy");
    if (!st) st = c->hip(hipStreamSynchronize(c->stream), "speed sync");
    if (st) return st;
    float vmax;
    std::memcpy(&vmax, &h_vmax, sizeof(float));
    const double cells = (double)vmax * in.cfg.dt / std::min(in.d.g.dx, in.d.g.dy);
    const double k = cells > 0 ? std::floor(in.d.tp.slack / cells) : 1e9;
    in.every = (int)std::max<double>(in.every_worst, std::min<double>(k, 3.0 * in.every_worst));
  }
  c->sort_every = 64;
  for (const Instance& other : c->inst) c->sort_every = std::min(c->sort_every, other.every);
  c->moves = c->sort_every;  // sort before the next particle pass
  c->phase = READY;
  return PIC_OK;
}

pic_status_t deposit_current(pic_ctx_t c) {
  if (!c) return PIC_ERR_INVALID_ARG;
  if (c->phase != READY) return c->fail(PIC_ERR_STATE, "deposit_current needs phase READY");
  pic_status_t st = particle_pass(c, 0);
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
  pic_status_t st = particle_pass(c, 1);
  if (st) return st;
  c->phase = READY;
  return PIC_OK;
}

// exported names stay out of internal calls: a call to a global symbol from
// inside the library could bind to another library's symbol of the same name
pic_status_t step(pic_ctx_t c, int32_t nsteps) { return run_steps(c, nsteps); }
pic_status_t step_batched(pic_ctx_t c, int32_t nsteps) { return run_steps(c, nsteps); }

pic_status_t pic_get_particles(pic_ctx_t c, double* out) {
  if (!c) return PIC_ERR_INVALID_ARG;
  if (c->phase == EMPTY) return c->fail(PIC_ERR_STATE, "no particles loaded");
  Instance& in = c->I();
  if (in.d.n > 0 && !out) return c->fail(PIC_ERR_INVALID_ARG, "out is NULL");
  auto pa = parts_of(c, in.d, c->cur);
  return c->hip(launch_get_particles(c->dtype, &pa, in.d.n, out, c->stream), "get_particles");
}

pic_status_t pic_set_particles(pic_ctx_t c, const double* src) {
  if (!c) return PIC_ERR_INVALID_ARG;
  if (c->phase == EMPTY) return c->fail(PIC_ERR_STATE, "no particles loaded");
  Instance& in = c->I();
  if (in.d.n > 0 && !src) return c->fail(PIC_ERR_INVALID_ARG, "in is NULL");
  // J is zero in both phases (consumed by the last field solve)
  if (c->phase != READY && c->phase != SOLVED) return c->fail(PIC_ERR_STATE, "set_particles needs phase READY or SOLVED");
  auto pa = parts_of(c, in.d, c->cur);
  c->order_tag = new_order_tag();
  c->from_sort = false;
  pic_status_t st = c->hip(launch_set_particles(c->dtype, &pa, in.d.n, src, in.d.g, c->stream), "set_particles");
  if (st) return st;
  c->moves = c->sort_every;  // re-sort before the next particle pass
  c->phase = READY;
  return PIC_OK;
}

pic_status_t pic_get_field(pic_ctx_t c, int32_t which, double* dst) {
  if (!c) return PIC_ERR_INVALID_ARG;
  if (!dst) return c->fail(PIC_ERR_INVALID_ARG, "dst is NULL");
  Instance& in = c->I();
  const size_t plane = (size_t)in.cfg.nx * in.cfg.ny;
  if (which == PIC_FIELD_J) {
    if (c->phase != DEPOSITED) return c->fail(PIC_ERR_STATE, "J is valid in phase DEPOSITED");
    const size_t nj = (size_t)j_planes(in.d.sc, 0) * plane;
    if (in.d.det)  // int64 at scale 2^qe_det
      return c->hip(launch_j_export(reinterpret_cast<const long long*>(in.d.J), dst, nj, in.d.det_unscale, c->stream),
                    "export J");
    return c->hip(hipMemcpyAsync(dst, in.d.J, nj * 8, hipMemcpyDeviceToDevice, c->stream), "copy J");
  }
  if (which == PIC_FIELD_MESH) {
    if (c->phase != SOLVED) return c->fail(PIC_ERR_STATE, "mesh fields are valid in phase SOLVED");
    if (c->dtype == PIC_F32) {
      // the step writes only the float32 copy: the float64 planes from the
      // solve's spectra (U is valid until the next solve)
      pic_status_t st = c->hip(launch_rows_c2r(c->d_desc, c->ninst(), c->nblk[BK_C2R], c->lds_c2r, c->stream,
                                               false, true),
                               "mesh field export");
      if (st) return st;
    }
    return c->hip(hipMemcpyAsync(dst, in.d.F64, 12 * plane * 8, hipMemcpyDeviceToDevice, c->stream),
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
  Instance& in = c->I();
  // the newest level is the one written by the last update: slots of s = nupd
  HistSlots hs = slots_of(c->hist, c->nupd);
  pic_status_t st = c->hip(launch_field_diag(in.d.H, in.d.g, in.d.sc, hs, c->d_diag, c->stream), "field diag");
  if (st) return st;
  auto pa = parts_of(c, in.d, c->cur);
  st = c->hip(launch_particle_diag(c->dtype, &pa, in.d.n, in.d.ph, c->d_diag + 16, c->stream), "particle diag");
  if (st) return st;
  std::vector<double> h(kDiagDoubles);
  st = c->hip(hipMemcpyAsync(h.data(), c->d_diag, h.size() * 8, hipMemcpyDeviceToHost, c->stream), "diag copy");
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

pic_status_t pic_set_dirk_tableau(pic_ctx_t c, int32_t stages, const double* A, const double* b,
                                  const double* cc) {
  if (!c) return PIC_ERR_INVALID_ARG;
  if (scheme_family(c->scheme) != PIC_SCHEME_DIRK2)
    return c->fail(PIC_ERR_UNSUPPORTED, "a DIRK tableau needs a DIRK scheme (PIC_SCHEME_DIRK2 or PIC_SCHEME_DIRK3)");
  if (!A || !b || !cc) return c->fail(PIC_ERR_INVALID_ARG, "A, b and c must be host arrays");
  const int ns = c->inst[0].d.sc.stages;
  if (stages != ns)
    return c->fail(PIC_ERR_INVALID_ARG, "the context's scheme has " + std::to_string(ns) +
                                            " stages (PIC_SCHEME_DIRK2: 2, PIC_SCHEME_DIRK3: 3)");
  if (c->phase == DEPOSITED || c->phase == SOLVED)
    return c->fail(PIC_ERR_STATE, "the tableau changes between steps only (phase READY or no particles yet)");
  double sb = 0;
  for (int i = 0; i < ns; ++i) {
    double row = 0;
    for (int j = 0; j < ns; ++j) {
      const double a = A[i * ns + j];
      if (!std::isfinite(a)) return c->fail(PIC_ERR_INVALID_ARG, "tableau entries must be finite");
      if (j > i && a != 0.0) return c->fail(PIC_ERR_INVALID_ARG, "A must be lower triangular (a DIRK)");
      row += a;
    }
    if (!(A[i * ns + i] > 0.0)) return c->fail(PIC_ERR_INVALID_ARG, "the diagonal of A must be positive");
    if (!std::isfinite(b[i]) || !std::isfinite(cc[i])) return c->fail(PIC_ERR_INVALID_ARG, "b and c must be finite");
    if (std::fabs(cc[i] - row) > 1e-12 * std::max(1.0, std::fabs(row)))
      return c->fail(PIC_ERR_INVALID_ARG, "c_i must equal the row sums of A");
    sb += b[i];
  }
  if (std::fabs(sb - 1.0) > 1e-12) return c->fail(PIC_ERR_INVALID_ARG, "the weights b must sum to one");
  for (auto& in : c->inst) {
    SchemeCoef& sc = in.d.sc;
    for (int i = 0; i < ns; ++i) {
      sc.dirkB[i] = b[i];
      sc.dirkC[i] = cc[i];
      for (int j = 0; j < ns; ++j) sc.dirkA[i][j] = A[i * ns + j];
    }
  }
  return c->upload_desc();
}

// byte offsets of one instance's parts inside a saved state
struct StateLayout {
  size_t parts, ids, start, cstart, work, nwork, hist, rb, fields, end;
};
// the mesh fields the gather reads (float32 contexts: the node-major copy;
// float64: the twelve planes), kept by states saved in phase SOLVED
static size_t field_state_bytes(const Instance& in) {
  const size_t plane = (size_t)in.cfg.nx * in.cfg.ny;
  return in.d.F32 ? 12 * plane * 4 : 12 * plane * 8;
}
static StateLayout state_layout(pic_ctx_t c, const Instance& in, size_t base) {
  StateLayout L{};
  const size_t es = c->dtype == PIC_F32 ? 4 : 8;
  const size_t cap = (size_t)in.cfg.max_particles;
  size_t o = base;
  auto take = [&](size_t bytes) {
    const size_t at = o;
    o = align_up(o + bytes);
    return at;
  };
  L.parts = take(11 * array_bytes(cap, es));
  L.ids = take(cap * 4);
  L.start = take(((size_t)in.d.tp.ntiles + 1) * 4);
  L.cstart = take((size_t)in.d.tp.ntiles * 4);
  L.work = take((size_t)in.d.tp.max_work * 16);
  L.nwork = take(4);
  L.hist = take((size_t)c->hist.nslots * in.L.plane_c * 16);
  L.rb = take(in.d.RB ? (size_t)in.cfg.nx * in.cfg.ny * 8 : 0);
  L.fields = take(field_state_bytes(in));
  L.end = o;
  return L;
}

static size_t state_header_bytes(pic_ctx_t c) { return align_up((size_t)(kStateHeaderWords + c->ninst()) * 8); }

size_t pic_state_bytes(pic_ctx_t c) {
  if (!c) return 0;
  size_t o = state_header_bytes(c);
  for (const auto& in : c->inst) o = state_layout(c, in, o).end;
  return o;
}

// the context's fingerprint in a saved state: the workspace layout and the
// configuration that fix what the bytes mean
static int64_t state_fingerprint(pic_ctx_t c) {
  uint64_t h = 1469598103934665603ull;
  auto mix = [&](uint64_t v) {
    h ^= v;
    h *= 1099511628211ull;
  };
  mix(c->ninst());
  for (const auto& in : c->inst) {
    const unsigned char* b = reinterpret_cast<const unsigned char*>(&in.cfg);
    for (size_t k = 0; k < sizeof(pic_config_t); ++k) mix(b[k]);
  }
  return (int64_t)(h & 0x7fffffffffffffffull);
}

// the segments of a state: (state offset, context address, bytes) for every
// instance, with n_i particles each; solved: also the mesh fields
static std::vector<std::array<size_t, 3>> state_segments(pic_ctx_t c, int cur, const std::vector<int64_t>& ns,
                                                         bool solved) {
  std::vector<std::array<size_t, 3>> seg;
  size_t o = state_header_bytes(c);
  const size_t es = c->dtype == PIC_F32 ? 4 : 8;
  for (int i = 0; i < c->ninst(); ++i) {
    const Instance& in = c->inst[i];
    const StateLayout L = state_layout(c, in, o);
    const InstDesc& d = in.d;
    const size_t n = (size_t)ns[i], ab = array_bytes((size_t)in.cfg.max_particles, es);
    for (int a = 0; a < 11; ++a) seg.push_back({L.parts + a * ab, (size_t)d.set[cur][a], n * es});
    seg.push_back({L.ids, (size_t)d.ids[cur], n * 4});
    seg.push_back({L.start, (size_t)d.tb.start, ((size_t)d.tp.ntiles + 1) * 4});
    seg.push_back({L.cstart, (size_t)d.tb.cstart, (size_t)d.tp.ntiles * 4});
    seg.push_back({L.work, (size_t)d.tb.work, (size_t)d.tp.max_work * 16});
    seg.push_back({L.nwork, (size_t)d.tb.nwork, 4});
    seg.push_back({L.hist, (size_t)d.H, (size_t)c->hist.nslots * in.L.plane_c * 16});
    if (d.RB) seg.push_back({L.rb, (size_t)d.RB, (size_t)in.cfg.nx * in.cfg.ny * 8});
    if (solved) seg.push_back({L.fields, d.F32 ? (size_t)d.F32 : (size_t)d.F64, field_state_bytes(in)});
    o = L.end;
  }
  return seg;
}

// copy the segments between the state buffer and the context, in launches of
// at most kCopyMax segments (one launch for a single-instance context)
static pic_status_t copy_segments(pic_ctx_t c, const std::vector<std::array<size_t, 3>>& seg, char* state,
                                  bool to_state) {
  size_t k = 0;  // next segment to copy
  while (k < seg.size()) {
    CopyList L{};
    uint64_t spans = 0;
    for (; k < seg.size() && L.count < kCopyMax; ++k) {
      const auto& g = seg[k];
      if (g[2] == 0) continue;
      char* sp = state + g[0];
      char* cp = reinterpret_cast<char*>(g[1]);
      if (((uintptr_t)sp | (uintptr_t)cp) & (g[2] >= 16 ? 15 : 3))
        return c->fail(PIC_ERR_HIP, "state segment misaligned");
      L.src[L.count] = to_state ? cp : sp;
      L.dst[L.count] = to_state ? sp : cp;
      L.bytes[L.count] = g[2];
      L.first[L.count] = spans;
      spans += (g[2] + kCopySpan - 1) / kCopySpan;
      L.count++;
    }
    if (!L.count) continue;
    L.first[L.count] = spans;
    if (spans > 0x7fffffffu) return c->fail(PIC_ERR_INVALID_ARG, "state copy larger than the grid allows");
    hipLaunchKernelGGL(k_copy_list, dim3((unsigned)spans), dim3(kCopyThreads), 0, c->stream, L);
    pic_status_t st = c->hip(hipGetLastError(), "state copy");
    if (st) return st;
  }
  return PIC_OK;
}

pic_status_t pic_save_state_h(pic_ctx_t c, void* dst, int64_t* header) {
  if (!c) return PIC_ERR_INVALID_ARG;
  if (!dst || ((uintptr_t)dst & (kAlign - 1))) return c->fail(PIC_ERR_INVALID_ARG, "dst must be a 256-byte aligned device pointer");
  if (c->phase != READY && c->phase != SOLVED) return c->fail(PIC_ERR_STATE, "save_state needs phase READY or SOLVED");
  const bool solved = c->phase == SOLVED;
  char* b = static_cast<char*>(dst);
  const int ni = c->ninst();
  std::vector<int64_t> ns(ni);
  for (int i = 0; i < ni; ++i) ns[i] = c->inst[i].d.n;
  // header: global words, then the particle counts (in launches of 16 words)
  std::vector<int64_t> words(kStateHeaderWords + ni, 0);
  const int64_t g[] = {(int64_t)kStateMagic, state_fingerprint(c), c->nupd, c->vflip, c->cur, c->moves,
                       c->stepped ? 1 : 0, (int64_t)pic_state_bytes(c), c->sort_every, (int64_t)c->order_tag,
                       c->from_sort ? 1 : 0, solved ? 1 : 0, c->adjoined ? 1 : 0};
  for (size_t k = 0; k < sizeof(g) / sizeof(g[0]); ++k) words[k] = g[k];
  for (int i = 0; i < ni; ++i) words[kStateHeaderWords + i] = ns[i];
  pic_status_t st = PIC_OK;
  for (size_t w0 = 0; w0 < words.size() && !st; w0 += kStateHeaderWords) {
    HeaderWords hw{};
    for (int k = 0; k < kStateHeaderWords && w0 + k < words.size(); ++k) hw.w[k] = words[w0 + k];
    const int cnt = (int)std::min<size_t>(kStateHeaderWords, words.size() - w0);
    hipLaunchKernelGGL(k_state_header, dim3(1), dim3(64), 0, c->stream, reinterpret_cast<int64_t*>(b) + w0, hw, cnt);
    st = c->hip(hipGetLastError(), "state header");
  }
  if (!st) st = copy_segments(c, state_segments(c, c->cur, ns, solved), b, true);
  if (!st && header) std::memcpy(header, words.data(), words.size() * sizeof(int64_t));
  return st;
}

pic_status_t pic_save_state(pic_ctx_t c, void* dst) { return pic_save_state_h(c, dst, nullptr); }

int32_t pic_state_header_words(pic_ctx_t c) { return c ? kStateHeaderWords + c->ninst() : 0; }

pic_status_t pic_load_state_h(pic_ctx_t c, const void* src, const int64_t* header) {
  if (!c) return PIC_ERR_INVALID_ARG;
  if (!src || ((uintptr_t)src & (kAlign - 1))) return c->fail(PIC_ERR_INVALID_ARG, "src must be a 256-byte aligned device pointer");
  const char* b = static_cast<const char*>(src);
  const int ni = c->ninst();
  std::vector<int64_t> h(kStateHeaderWords + ni);
  pic_status_t st = PIC_OK;
  if (header) {  // the caller's copy from pic_save_state_h: no read, no synchronisation
    std::memcpy(h.data(), header, h.size() * sizeof(int64_t));
  } else {
    st = c->hip(hipMemcpyAsync(h.data(), b, h.size() * 8, hipMemcpyDeviceToHost, c->stream), "state header read");
    if (!st) st = c->hip(hipStreamSynchronize(c->stream), "state header sync");
    if (st) return st;
  }
  if (h[0] != (int64_t)kStateMagic || h[1] != state_fingerprint(c) || h[7] != (int64_t)pic_state_bytes(c))
    return c->fail(PIC_ERR_INVALID_ARG, "src is not a state saved by a context of this configuration");
  std::vector<int64_t> ns(h.begin() + kStateHeaderWords, h.end());
  for (int i = 0; i < ni; ++i)
    if (ns[i] < 0 || ns[i] > c->inst[i].cfg.max_particles)
      return c->fail(PIC_ERR_INVALID_ARG, "src holds a particle count beyond the capacity");
  const int cur = (int)h[4];
  if (cur != 0 && cur != 1) return c->fail(PIC_ERR_INVALID_ARG, "src holds an invalid particle set index");
  if (h[11] != 0 && h[11] != 1) return c->fail(PIC_ERR_INVALID_ARG, "src holds an invalid phase");
  const bool solved = h[11] == 1;
  st = copy_segments(c, state_segments(c, cur, ns, solved), const_cast<char*>(b), false);
  if (st) {
    c->phase = EMPTY;
    return st;
  }
  bool counts_changed = false;
  for (int i = 0; i < ni; ++i) {
    counts_changed = counts_changed || c->inst[i].d.n != ns[i];
    c->inst[i].d.n = ns[i];
  }
  c->nupd = h[2];
  c->vflip = (int)h[3];
  c->cur = cur;
  c->moves = (int)h[5];
  c->stepped = h[6] != 0;
  c->sort_every = (int)std::min<int64_t>(std::max<int64_t>(h[8], 1), 64);
  c->order_tag = (uint64_t)h[9];
  c->from_sort = h[10] != 0;
  c->adjoined = h[12] != 0;
  c->phase = solved ? SOLVED : READY;
  // the device descriptors change only with the particle counts
  return counts_changed ? c->upload_desc() : PIC_OK;
}

pic_status_t pic_load_state(pic_ctx_t c, const void* src) { return pic_load_state_h(c, src, nullptr); }

pic_status_t pic_diagnostics_all(pic_ctx_t c, double* out) {
  if (!c) return PIC_ERR_INVALID_ARG;
  if (!out) return c->fail(PIC_ERR_INVALID_ARG, "out is NULL");
  const int n = c->ninst();
  if (n > kDiagAllMax)
    return c->fail(PIC_ERR_INVALID_ARG, "pic_diagnostics_all covers at most " + std::to_string(kDiagAllMax) +
                                            " instances (the context holds " + std::to_string(n) + ")");
  const HistSlots hs = slots_of(c->hist, c->nupd);
  for (int i = 0; i < n; ++i) {
    const InstDesc& d = c->inst[i].d;
    double* p = c->d_scratch + (size_t)i * kDiagDoubles;
    pic_status_t st = c->hip(launch_field_diag(d.H, d.g, d.sc, hs, p, c->stream), "field diag");
    if (st) return st;
    auto pa = parts_of(c, d, c->cur);
    st = c->hip(launch_particle_diag(c->dtype, &pa, d.n, d.ph, p + 16, c->stream), "particle diag");
    if (st) return st;
  }
  hipLaunchKernelGGL(k_diag_finalize, dim3(n), dim3(64), 0, c->stream, c->d_scratch, n, out);
  return c->hip(hipGetLastError(), "diag finalize");
}

// ---------------------------------------------------------------------------
// discrete adjoint (float64 BDF-k, one instance, PIC_FLAG_ADJOINT)

static pic_status_t adjoint_check(pic_ctx_t c, bool need_ready) {
  if (c->ninst() != 1) return c->fail(PIC_ERR_UNSUPPORTED, "the adjoint runs on single-instance contexts");
  if (!(c->I().cfg.flags & PIC_FLAG_ADJOINT))
    return c->fail(PIC_ERR_UNSUPPORTED, "the adjoint needs a context created with PIC_FLAG_ADJOINT");
  if (c->dtype != PIC_F64 || c->scheme != PIC_SCHEME_BDF || c->degree > 3)
    return c->fail(PIC_ERR_UNSUPPORTED,
                   "the adjoint supports float64 particles, the BDF-k stepper and spline degrees 1..3");
  if (need_ready && c->phase != READY) return c->fail(PIC_ERR_STATE, "adjoint_seed_energy and step_adjoint need phase READY");
  if (c->phase == EMPTY) return c->fail(PIC_ERR_STATE, "no particles loaded");
  return PIC_OK;
}

pic_status_t adjoint_seed_energy(pic_ctx_t c, double scale, double* lam_hist) {
  if (!c) return PIC_ERR_INVALID_ARG;
  pic_status_t st = adjoint_check(c, true);
  if (st) return st;
  if (!lam_hist) return c->fail(PIC_ERR_INVALID_ARG, "lam_hist is NULL");
  Instance& in = c->I();
  return c->hip(launch_adj_seed_energy(in.d.H, in.d.g, in.d.sc, slots_of(c->hist, c->nupd), scale, lam_hist,
                                       c->hist.nexport, c->stream),
                "adjoint seed");
}

pic_status_t pic_adjoint_set_particles(pic_ctx_t c, const double* lam) {
  if (!c) return PIC_ERR_INVALID_ARG;
  pic_status_t st = adjoint_check(c, false);
  if (st) return st;
  Instance& in = c->I();
  st = c->hip(launch_lam_set(in.d.n, lam, in.d.LAM, in.cfg.max_particles, in.d.LIDS, in.d.ids[c->cur], c->stream),
              "adjoint set");
  c->lam_n = st ? -1 : in.d.n;
  // NULL: zero in the current slot order; else original order (checked on the device)
  c->lam_tag = lam ? 0 : c->order_tag;
  return st;
}

pic_status_t pic_adjoint_get_particles(pic_ctx_t c, double* lam) {
  if (!c) return PIC_ERR_INVALID_ARG;
  pic_status_t st = adjoint_check(c, false);
  if (st) return st;
  Instance& in = c->I();
  if (in.d.n > 0 && !lam) return c->fail(PIC_ERR_INVALID_ARG, "lam is NULL");
  if (c->lam_n != in.d.n) return c->fail(PIC_ERR_STATE, "no particle adjoint held for the loaded particles");
  return c->hip(launch_lam_get(in.d.n, in.d.LAM, in.cfg.max_particles, in.d.LIDS, lam, c->stream), "adjoint get");
}

pic_status_t step_adjoint(pic_ctx_t c, double* lam, double* lam_hist) {
  if (!c) return PIC_ERR_INVALID_ARG;
  pic_status_t st = adjoint_check(c, false);
  if (st) return st;
  if (c->phase != READY && c->phase != SOLVED) return c->fail(PIC_ERR_STATE, "step_adjoint needs phase READY or SOLVED");
  if (c->phase == SOLVED && c->adjoined)
    return c->fail(PIC_ERR_STATE, "step_adjoint already ran on this state (load the next one)");
  Instance& in = c->I();
  if (!lam_hist) return c->fail(PIC_ERR_INVALID_ARG, "lam_hist must be a device pointer");
  if (lam) {
    st = pic_adjoint_set_particles(c, lam);
    if (st) return st;
  } else if (c->lam_n != in.d.n) {
    return c->fail(PIC_ERR_STATE, "lam is NULL and no particle adjoint is held for the loaded particles");
  }
  // phase READY: recompute x^{n+1}, J^{n+1} and the level-(n+1) fields from
  // the loaded state, without the sort the forward may have made before this
  // deposit when the loaded order comes from a sort (its chunks hold every
  // particle): the next state is loaded over this one anyway, and a sort here
  // would cost the scatter and two permutations of the held adjoint (into the
  // new order and back to the next loaded state's).  Phase SOLVED: the
  // context already holds them (a state saved after deposit_current and
  // field_solve)
  if (c->phase == READY) {
    st = particle_pass(c, 0, !c->from_sort);
    if (!st) st = do_solve(c);
  }
  const InstDesc* D = c->d_desc;
  const int nx = in.cfg.nx, ny = in.cfg.ny;
  const StepArgs sa = c->sargs();
  const int64_t ls = in.cfg.max_particles;
  // the held adjoint follows the order of the set the passes run on: checked
  // (and permuted) on the device unless it already follows this order's tag
  if (!st && c->lam_tag != c->order_tag) {
    st = c->hip(launch_lam_follow(in.d.n, in.d.ids[c->cur], in.d.LAM, in.d.LAM2, ls, in.d.LIDS, in.d.LINV,
                                  in.d.LFLAG, c->stream),
                "adjoint order");
    if (!st) c->lam_tag = c->order_tag;
  }
  // the cell-sorted passes when the forward is sorted and the windows fit in LDS
  int max_lds = 0, dev = 0;
  (void)hipGetDevice(&dev);
  (void)hipDeviceGetAttribute(&max_lds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev);
  const size_t lds_push = adj_tiled_lds_bytes(in.d.tp, true), lds_dep = adj_tiled_lds_bytes(in.d.tp, false);
  const bool tiled = c->sorted && lds_push <= (size_t)max_lds;
  const int geo = tiled_geometry(in.d.tp), nwb = c->nblk[BK_WORK];
  if (!st)
    st = c->hip(tiled ? launch_adj_tiled(true, c->degree, geo, D, nwb, lds_push, sa, in.d.LAM, ls, c->stream)
                      : launch_adj_push(c->degree, D, in.d.n, sa, in.d.LAM, ls, c->stream),
                "adjoint push");
  if (!st) st = c->hip(launch_rows_r2c(D, 1, 11 * (ny / in.d.R_r2c), c->lds_r2c, c->stream, true), "adjoint rows_r2c");
  if (!st) st = c->hip(launch_adj_columns(in.cfg.bdf_order, D, nx / 2 + 1, c->lds_adj_col, lam_hist, c->stream), "adjoint columns");
  if (!st) st = c->hip(launch_rows_c2r(D, 1, 2 * (ny / in.d.R_c2r), c->lds_c2r, c->stream, true), "adjoint rows_c2r");
  if (!st)
    st = c->hip(tiled ? launch_adj_tiled(false, c->degree, geo, D, nwb, lds_dep, sa, in.d.LAM, ls, c->stream)
                      : launch_adj_deposit(c->degree, D, in.d.n, sa, in.d.LAM, ls, c->stream),
                "adjoint deposit");
  if (!st && lam) st = pic_adjoint_get_particles(c, lam);
  if (st) {
    c->lam_n = -1;
    c->lam_tag = 0;
  }
  c->phase = st ? EMPTY : SOLVED;
  c->adjoined = !st;
  return st;
}

pic_status_t adjoint_initial(pic_ctx_t c, const double* P0, double* lam) {
  if (!c) return PIC_ERR_INVALID_ARG;
  pic_status_t st = adjoint_check(c, false);
  if (st) return st;
  Instance& in = c->I();
  if (in.d.n > 0 && (!P0 || !lam)) return c->fail(PIC_ERR_INVALID_ARG, "P0 and lam must be device pointers");
  return c->hip(launch_adj_initial(in.d.n, P0, in.d.ph, lam, c->stream), "adjoint initial");
}

int32_t pic_graph_period(pic_ctx_t c) {
  if (!c || !c->use_graphs || !c->sorted || c->timing) return 0;
  return graph_period(c);
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
