// Field solve on the periodic grid: R2C FFT of J, continuity, the stepper's
// modified-Helmholtz update in Fourier space, spectral gradients and C2R FFTs.
//
// Paper: the update formulas of Sec. 3.1 (implicit CDF-2, Crank-Nicolson form
// with alpha = sqrt(2)/(c dt)), Sec. 3.2 (BDF-k, L^{-1} update with C = a*a),
// Sec. 3.3 (s-stage DIRK on the first-order system, stage operators
// L_i = I - Laplacian/alpha_i^2, alpha_i = 1/(h a_ii c)); continuity in each
// stepper's form (Algorithm 1, third step); spectral derivatives (Sec. 4.1).
//
// Data flow (x fastest in real space, complex128 spectra):
//   J   [3][ny][nx]        real, consumed (zeroed) by k_rows_r2c; naive charge
//                          mode: a fourth plane, the deposited rho, reset to the
//                          ion background instead of zero
//   T   [3][nxh][ny]       x-transformed J (naive: [4], rho last), transposed so
//                          columns are contiguous
//   H   [slot][nxh][ny]    spectral history (ring slots chosen by the host)
//   U   [8][nxh][ny]       y-inverse-transformed phi~, d_y phi~, A, d_y A
//   F   [12][ny][nx]       real mesh fields for the gather (float64); the float32
//                          copy is node-major [ny][nx][12]
// Reading of the Nyquist mode (the paper is silent): the first-derivative
// symbol is zero at index n/2 of each axis and the Laplacian is built from the
// same symbols, so div(grad) equals the Laplacian exactly.
#include "fft_lds.h"

#include <algorithm>
#include <cmath>

namespace pic {

namespace {


// ---------------------------------------------------------------------------
// rows: R real rows (R even) of one J component -> R/2 complex FFTs along x.
// Flattened over instances: local block = component * ceil(ny/R) + row group;
// rows past ny in the last group (ny not a multiple of R) read as zero and are
// not written.
// adj: the same transform of the 11 adjoint mesh fields LF into LS.
__global__ void __launch_bounds__(256) k_rows_r2c(const InstDesc* __restrict__ D, int ninst, int adj) {
  extern __shared__ double2 sm[];
  // neighbouring row groups on one XCD: each writes R of the ny values of a
  // spectrum column, so the groups that fill one cache line share its L2
  const int bb = xcd_contiguous(blockIdx.x, gridDim.x);
  const int ii = find_inst(D, ninst, BK_R2C, bb);
  const InstDesc& d = D[ii];
  const GridP g = d.g;
  const int R = d.R_r2c, ngr = (g.ny + R - 1) / R;
  const int lb = bb - d.blk[BK_R2C];
  const int c = lb / ngr, y0 = (lb - c * ngr) * R;
  const int nr = min(R, g.ny - y0);  // rows of this group
  const gptr<double> Jc = gp((adj ? d.LF : d.J) + (size_t)c * g.nx * g.ny);
  // the naive mode's rho plane restarts from the ion background
  const gptr<const double> reset = gp((const double*)((!adj && c == 3) ? d.RB : nullptr));
  const bool det = !adj && d.det;
  const GC2 T = gc2(adj ? d.LS : d.T);
  const int N = g.nx, B = R >> 1;
  double2* a = sm;
  double2* b = sm + B * N;
  double2* tws = sm + R * N;  // twiddles staged in LDS
  for (int t = threadIdx.x; t < N; t += blockDim.x) tws[t] = gc2(d.twx)[t];
  for (int t = threadIdx.x; t < B * N; t += blockDim.x) {
    const int r = t / N, x = t - r * N;
    const size_t i0 = (size_t)(y0 + 2 * r) * N + x, i1 = i0 + N;
    const bool h0 = 2 * r < nr, h1 = 2 * r + 1 < nr;
    if (det) {  // deterministic deposit: int64 sums at scale 2^qe_det
      const gptr<const long long> Jq = reinterpret_cast<gptr<const long long>>(Jc);
      a[t] = make_double2(h0 ? (double)Jq[i0] * d.det_unscale : 0.0, h1 ? (double)Jq[i1] * d.det_unscale : 0.0);
    } else {
      a[t] = make_double2(h0 ? Jc[i0] : 0.0, h1 ? Jc[i1] : 0.0);
    }
    // consumed: ready for the next deposit (or adjoint scatter)
    if (h0) Jc[i0] = reset ? reset[i0] : 0.0;
    if (h1) Jc[i1] = reset ? reset[i1] : 0.0;
  }
  __syncthreads();
  const double2* res = fft_lds<false>(a, b, N, B, tws);
  // split the two real transforms: X = (Z_k + conj Z_{N-k})/2, Y = (Z_k - conj Z_{N-k})/(2i)
  for (int t = threadIdx.x; t < g.nxh * R; t += blockDim.x) {
    const int k = t / R, rr = t - k * R, r = rr >> 1;
    if (rr >= nr) continue;
    const double2 zk = res[r * N + k];
    const double2 zn = cconj(res[r * N + (k ? N - k : 0)]);
    double2 o;
    if ((rr & 1) == 0) {
      o = cscale(cadd(zk, zn), 0.5);
    } else {
      const double2 dd = csub(zk, zn);
      o = make_double2(0.5 * dd.y, -0.5 * dd.x);
    }
    T[((size_t)c * g.nxh + k) * g.ny + y0 + rr] = o;
  }
}

// ---------------------------------------------------------------------------
// columns: four blocks per kx, one per output.  Forward y-FFT of the J
// columns, the stepper's update for every ky of this column, and inverse
// y-FFTs of the part's two outputs (scaled by 1/(nx ny)).  Part 0 updates
// rho and phi (DIRK: and v_phi) from the forward y-FFTs of J_x and J_y (the
// divergence); part 1 + l updates A_l (DIRK: and v_A,l) from the forward
// y-FFT of J_l.  Each part inverse-transforms its two outputs (phi~ and
// d_y phi~, or A_l and d_y A_l).  The history terms of the update do not
// depend on J^{n+1}: they are loaded (BDF-k: summed) before the forward
// transform, so their loads overlap it.  Parts share no written state: DIRK's
// J^n history is a ring of two levels, read at J[0] by parts 0 and 1 + l and
// written at J_new by part 1 + l only.
constexpr int kColParts = 4;
constexpr int kMaxStages = 3;  // DIRK stages: loops over them unrolled to this bound (registers, not scratch)
// modes per thread: 256 threads up to ny = 512, 512 threads above (ny <= 1024);
// two modes keep the DIRK update's per-mode values within a register budget
// that admits three waves per SIMD
constexpr int kColMaxModes = 2;

template <int SCHEME, int K>
__global__ void __launch_bounds__(512) k_columns_split(const InstDesc* __restrict__ D, int ninst, HistSlots hs) {
  // LDS: [0, N) the scaled output column; [N, 5N) work (two ping-pong pairs
  // of two columns); then the N twiddles (ny <= 512); then, for sub-stepped
  // DIRK currents, the transformed stage columns (two per stage)
  extern __shared__ double2 sm[];
  // the four parts of one column on one XCD: parts 0 and 1 + l read the same
  // transformed J columns, which then come from one L2
  const int bb = xcd_contiguous(blockIdx.x, gridDim.x);
  const int ii = find_inst(D, ninst, BK_COL, bb);
  const InstDesc& d = D[ii];
  const GridP g = d.g;
  const SchemeCoef sc = d.sc;
  const int lb = bb - d.blk[BK_COL];
  const int kx = lb / kColParts, part = lb - kx * kColParts;
  const int N = g.ny, tid = threadIdx.x, nth = blockDim.x;
  const GC2 T = gc2(d.T);
  const GC2 H = gc2(d.H);
  const GC2 U = gc2(d.U);
  const size_t plane = (size_t)g.nxh * N;
  double2* store = sm;
  double2* wk = sm + N;
  const double2* tws = d.twy;
  if (N <= 512) {
    double2* t_lds = sm + 5 * N;
    for (int i = tid; i < N; i += nth) t_lds[i] = gc2(d.twy)[i];
    tws = t_lds;
  }
  double2* stg = sm + (N <= 512 ? 6 : 5) * N;
  // sub-stepped DIRK stages (their currents sit at T components 3 i .. 3 i + 2)
  const int nst = SCHEME == PIC_SCHEME_DIRK2 && sc.substep ? sc.stages : 0;
  // part 0 transforms J_x, J_y (the divergence), or in the naive mode the
  // deposited rho (component 3); part 1 + l transforms J_l
  const bool naive_rho = part == 0 && d.naive;
  const int ncol = part == 0 && !naive_rho ? 2 : 1;
  const int c0 = part == 0 ? (naive_rho ? 3 : 0) : part - 1;
  for (int i = tid; i < ncol * N; i += nth) {
    const int c = i / N, y = i - c * N;
    wk[i] = T[((size_t)(c0 + c) * g.nxh + kx) * N + y];
  }
  // history terms of this thread's modes ky = tid + m * nth
  auto at = [&](int slot, int ky) -> decltype(auto) { return H[(size_t)slot * plane + (size_t)kx * N + ky]; };
  double2 h0[kColMaxModes], h1[kColMaxModes], h2[kColMaxModes], h3[kColMaxModes], h4[kColMaxModes];
#pragma unroll
  for (int m = 0; m < kColMaxModes; ++m) {
    const int ky = tid + m * nth;
    h0[m] = h1[m] = h2[m] = h3[m] = h4[m] = make_double2(0.0, 0.0);
    if (ky >= N) continue;
    if (SCHEME == PIC_SCHEME_BDF) {
      if (part == 0) {
        // sum_j a_j rho^{n+1-j} (continuity only) and sum_i C_i phi^{n+1-i}
        if (!naive_rho) {
#pragma unroll
          for (int j = 1; j <= K; ++j) h0[m] = cadd(h0[m], cscale(at(hs.rho[j - 1], ky), sc.a[j]));
        }
#pragma unroll
        for (int i = 1; i <= 2 * K; ++i) h1[m] = cadd(h1[m], cscale(at(hs.phi[i - 1], ky), sc.Cn[i]));
      } else {
#pragma unroll
        for (int i = 1; i <= 2 * K; ++i) h0[m] = cadd(h0[m], cscale(at(hs.A[i - 1] + c0, ky), sc.Cn[i]));
      }
    } else if (SCHEME == PIC_SCHEME_CDF2) {
      if (part == 0) {
        h0[m] = at(hs.rho[0], ky);
        h1[m] = at(hs.rho[1], ky);
        h2[m] = at(hs.phi[0], ky);
        h3[m] = at(hs.phi[1], ky);
      } else {
        // J^{n-1} for the implicit form's averaged source, J^n for the others
        h0[m] = at(hs.A[0] + c0, ky);
        h1[m] = at(hs.A[1] + c0, ky);
        h2[m] = at(hs.J[sc.form == 0 ? 1 : 0] + c0, ky);
      }
    } else {  // DIRK: u^n, v^n of the part's wave component, and J^n for interpolated stages
      if (part == 0) {
        h0[m] = at(hs.rho[0], ky);
        h1[m] = at(hs.phi[0], ky);
        h2[m] = at(hs.vphi, ky);
        if (!nst && !naive_rho) {
          h3[m] = at(hs.J[0], ky);
          h4[m] = at(hs.J[0] + 1, ky);
        }
      } else {
        h0[m] = at(hs.A[0] + c0, ky);
        h1[m] = at(hs.vA + c0, ky);
        if (!nst) h2[m] = at(hs.J[0] + c0, ky);
      }
    }
  }
  __syncthreads();
  const double2* Jh;
  if (nst) {
    // stage by stage into the stage region (stage i at stg + i * ncol * N)
    for (int st = 0; st < nst; ++st) {
      if (st > 0) {
        for (int i = tid; i < ncol * N; i += nth) {
          const int c = i / N, y = i - c * N;
          wk[i] = T[((size_t)(3 * st + c0 + c) * g.nxh + kx) * N + y];
        }
        __syncthreads();
      }
      const double2* r = fft_lds<false>(wk, wk + 2 * N, N, ncol, tws);
      for (int i = tid; i < ncol * N; i += nth) stg[st * ncol * N + i] = r[i];
      __syncthreads();
    }
    Jh = stg;
  } else {
    Jh = fft_lds<false>(wk, wk + 2 * N, N, ncol, tws);
  }
  const double kxs = kx_sym(kx, g);
  const double scale = 1.0 / ((double)g.nx * g.ny);
#pragma unroll
  for (int m = 0; m < kColMaxModes; ++m) {
    const int ky = tid + m * nth;
    if (ky >= N) continue;
    const double kys = ky_sym(ky, g);
    const double Lh = 1.0 + (kxs * kxs + kys * kys) * sc.inv_alpha2;
    double2 out;
    // i k . V
    auto divv = [&](double2 X, double2 Y) { return mul_i(make_double2(kxs * X.x + kys * Y.x, kxs * X.y + kys * Y.y)); };
    if (SCHEME == PIC_SCHEME_DIRK2) {
      // Sec. 3.3: s-stage DIRK on (u, v)' = (v, c^2 (S + Lap u)), Lap = -kappa,
      // one scalar wave component per part
      const double h = sc.dt, c2 = sc.c * sc.c, kappa = kxs * kxs + kys * kys;
      const int ns = sc.stages;
      auto advance = [&](double2& u, double2& v, const double2* S) {
        double2 ku[kMaxStages], kv[kMaxStages];
#pragma unroll
        for (int i = 0; i < kMaxStages; ++i) {
          if (i >= ns) break;
          double2 U = u, V = v;
#pragma unroll
          for (int j = 0; j < i; ++j) {
            U = cadd(U, cscale(ku[j], h * sc.dirkA[i][j]));
            V = cadd(V, cscale(kv[j], h * sc.dirkA[i][j]));
          }
          const double hai = h * sc.dirkA[i][i];
          const double Li = 1.0 + hai * hai * c2 * kappa;
          const double2 src = csub(S[i], cscale(U, kappa));  // S + Lap U
          ku[i] = cdivr(cadd(V, cscale(src, hai * c2)), Li);
          kv[i] = cdivr(csub(cscale(src, c2), cscale(V, hai * c2 * kappa)), Li);
        }
#pragma unroll
        for (int i = 0; i < kMaxStages; ++i) {
          if (i >= ns) break;
          u = cadd(u, cscale(ku[i], h * sc.dirkB[i]));
          v = cadd(v, cscale(kv[i], h * sc.dirkB[i]));
        }
      };
      double2 S[kMaxStages];
      if (part == 0) {
        const double2 rho_n = h0[m];
        double2 rho = rho_n, rst[kMaxStages];
        if (nst) {
          // sub-stepped currents: rho^(i) are the RK stage values of the
          // continuity equation, rho^{n+1} its final stage
          double2 dv[kMaxStages];
#pragma unroll
          for (int i = 0; i < kMaxStages; ++i) {
            if (i >= ns) break;
            dv[i] = divv(Jh[(2 * i) * N + ky], Jh[(2 * i + 1) * N + ky]);
            rho = csub(rho, cscale(dv[i], h * sc.dirkB[i]));
          }
#pragma unroll
          for (int i = 0; i < kMaxStages; ++i) {
            if (i >= ns) break;
            rst[i] = rho_n;
#pragma unroll
            for (int j = 0; j <= i; ++j) rst[i] = csub(rst[i], cscale(dv[j], h * sc.dirkA[i][j]));
          }
        } else {
          if (naive_rho) {
            rho = Jh[ky];  // naive comparison: the deposited rho^{n+1}
          } else {
            const double2 J0 = Jh[ky], J1 = Jh[N + ky];
#pragma unroll
            for (int i = 0; i < kMaxStages; ++i) {
              if (i >= ns) break;
              const double2 X = cadd(cscale(h3[m], 1.0 - sc.dirkC[i]), cscale(J0, sc.dirkC[i]));
              const double2 Y = cadd(cscale(h4[m], 1.0 - sc.dirkC[i]), cscale(J1, sc.dirkC[i]));
              rho = csub(rho, cscale(divv(X, Y), h * sc.dirkB[i]));
            }
          }
#pragma unroll
          for (int i = 0; i < kMaxStages; ++i)
            if (i < ns) rst[i] = cadd(cscale(rho_n, 1.0 - sc.dirkC[i]), cscale(rho, sc.dirkC[i]));
        }
#pragma unroll
        for (int i = 0; i < kMaxStages; ++i)
          if (i < ns) S[i] = cscale(rst[i], 1.0 / sc.eps0);
        double2 u = h1[m], v = h2[m];
        advance(u, v, S);
        at(hs.rho_new, ky) = rho;
        at(hs.phi_new, ky) = u;
        at(hs.vphi, ky) = v;
        out = u;
      } else {
        double2 keep = make_double2(0.0, 0.0);
#pragma unroll
        for (int i = 0; i < kMaxStages; ++i) {
          if (i >= ns) break;
          // stage current: sub-stepped, or interpolated between J^n and J^{n+1}
          const double2 Ji = nst ? Jh[i * N + ky]
                                 : cadd(cscale(h2[m], 1.0 - sc.dirkC[i]), cscale(Jh[ky], sc.dirkC[i]));
          S[i] = cscale(Ji, sc.mu0);
          keep = cadd(keep, cscale(Ji, sc.dirkB[i]));
        }
        // J history: sum_i b_i J^(i) when sub-stepped, else J^{n+1}
        if (!nst) keep = Jh[ky];
        double2 u = h0[m], v = h1[m];
        advance(u, v, S);
        at(hs.A_new + c0, ky) = u;
        at(hs.vA + c0, ky) = v;
        at(hs.J_new + c0, ky) = keep;
        out = u;
      }
    } else if (part == 0) {
      const double2 J0 = Jh[ky], J1 = naive_rho ? J0 : Jh[N + ky];
      const double2 divJ = divv(J0, J1);  // i k . J
      if (SCHEME == PIC_SCHEME_BDF) {
        // continuity: sum_j a_j rho^{n+1-j} + dt div J^{n+1} = 0 (naive: the deposited rho)
        const double2 rho = naive_rho ? J0 : cscale(cadd(cscale(divJ, sc.dt), h0[m]), -1.0 / sc.a[0]);
        const double2 phi = cdivr(csub(cscale(rho, sc.inv_alpha2 / sc.eps0), h1[m]), Lh);
        at(hs.rho_new, ky) = rho;
        at(hs.phi_new, ky) = phi;
        out = phi;
      } else {
        // rho^{n+3/2} from the staggered continuity equation; h0..h3 =
        // rho^{n+1/2}, rho^{n-1/2}, phi^{n+1/2}, phi^{n-1/2}
        const double2 rho = csub(h0[m], cscale(divJ, sc.dt));
        double2 phi;
        if (sc.form == 0) {  // implicit: sources averaged over n+3/2 and n-1/2
          const double2 rhs = cadd(cscale(h2[m], 2.0), cscale(cadd(rho, h1[m]), sc.inv_alpha2 / sc.eps0));
          phi = csub(cdivr(rhs, Lh), h3[m]);
        } else if (sc.form == 1) {  // semi-implicit: source rho^{n+1/2}
          const double2 rhs = cadd(cscale(h2[m], 2.0), cscale(h0[m], 2.0 * sc.inv_alpha2 / sc.eps0));
          phi = csub(cdivr(rhs, Lh), h3[m]);
        } else {  // explicit: 2 phi - phi_old + c^2 dt^2 (Lap phi + rho/eps0), c^2 dt^2 = 2/alpha^2
          const double kap = kxs * kxs + kys * kys;
          phi = cadd(csub(cscale(h2[m], 2.0), h3[m]),
                     cscale(csub(cscale(h0[m], 1.0 / sc.eps0), cscale(h2[m], kap)), 2.0 * sc.inv_alpha2));
        }
        at(hs.rho_new, ky) = rho;
        at(hs.phi_new, ky) = phi;
        out = cscale(cadd(phi, h2[m]), 0.5);
      }
    } else {
      const double2 Jl = Jh[ky];
      if (SCHEME == PIC_SCHEME_BDF) {
        const double2 A = cdivr(csub(cscale(Jl, sc.mu0 * sc.inv_alpha2), h0[m]), Lh);
        at(hs.A_new + c0, ky) = A;
        out = A;
      } else {
        // h0, h1, h2 = A^n, A^{n-1}, and J^{n-1} (implicit) or J^n
        double2 A;
        if (sc.form == 0) {
          const double2 r = cadd(cscale(h0[m], 2.0), cscale(cadd(Jl, h2[m]), sc.mu0 * sc.inv_alpha2));
          A = csub(cdivr(r, Lh), h1[m]);
        } else if (sc.form == 1) {
          const double2 r = cadd(cscale(h0[m], 2.0), cscale(h2[m], 2.0 * sc.mu0 * sc.inv_alpha2));
          A = csub(cdivr(r, Lh), h1[m]);
        } else {
          const double kap = kxs * kxs + kys * kys;
          A = cadd(csub(cscale(h0[m], 2.0), h1[m]),
                   cscale(csub(cscale(h2[m], sc.mu0), cscale(h0[m], kap)), 2.0 * sc.inv_alpha2));
        }
        at(hs.A_new + c0, ky) = A;
        at(hs.J_new + c0, ky) = Jl;
        out = A;
      }
    }
    store[ky] = cscale(out, scale);
  }
  __syncthreads();
  // outputs: the field and its y derivative (G0, G1 or G(2+l), G(5+l))
  for (int i = tid; i < 2 * N; i += nth) {
    const int q = i / N, ky = i - q * N;
    const double2 v = store[ky];
    wk[i] = q ? mul_i(cscale(v, ky_sym(ky, g))) : v;
  }
  __syncthreads();
  const double2* res = fft_lds<true>(wk, wk + 2 * N, N, 2, tws);
  const int g0 = part == 0 ? 0 : 2 + c0, g1 = part == 0 ? 1 : 5 + c0;
  for (int i = tid; i < 2 * N; i += nth) {
    const int q = i / N, y = i - q * N;
    U[((size_t)(q ? g1 : g0) * g.nxh + kx) * N + y] = res[i];
  }
}

// ---------------------------------------------------------------------------
// rows C2R: R rows of one output pair (two real fields from one complex FFT).
// Pair p of the 12 mesh fields and the U column (and whether it is multiplied
// by i kx) each is made from:
//   0 d_x phi = ikx G0   1 d_y phi = G1   2 Ax = G2   3 Ay = G3   4 Az = G4
//   5 d_x Ax = ikx G2    6 d_x Ay = ikx G3   7 d_x Az = ikx G4
//   8 d_y Ax = G5        9 d_y Ay = G6      10 d_y Az = G7     11 phi~ = G0
__constant__ int kSrcG[12] = {0, 1, 2, 3, 4, 2, 3, 4, 5, 6, 7, 0};
__constant__ int kMulKx[12] = {1, 0, 0, 0, 0, 1, 1, 1, 0, 0, 0, 0};

//
// adj: the three columns LS[0..2] of the adjoint solve to the real fields LJ
// (pairs (0, 1) and (2, -); no kx factor).
// f64out: also write the float64 planes (always for float64 particles and the
// adjoint; float32 contexts read only the node-major float32 copy, and their
// float64 planes are written on demand for the mesh-field export)
__global__ void __launch_bounds__(256) k_rows_c2r(const InstDesc* __restrict__ D, int ninst, int adj, int f64out) {
  extern __shared__ double2 sm[];
  // the pairs of one row group in consecutive blocks, and neighbouring blocks
  // on one XCD: the six pairs of a row group fill each node's record (and
  // neighbouring row groups read one cache line of a spectrum column) through
  // one L2
  const int bb = xcd_contiguous(blockIdx.x, gridDim.x);
  const int ii = find_inst(D, ninst, BK_C2R, bb);
  const InstDesc& d = D[ii];
  const GridP g = d.g;
  const int R = d.R_c2r;
  const int np = adj ? 2 : 6;  // output pairs per row group
  const int lb = bb - d.blk[BK_C2R];
  const int rg = lb / np, pr = lb - rg * np, y0 = rg * R;
  const int nr = min(R, g.ny - y0);  // rows of this group (the last may be partial)
  const GC2 U = gc2(adj ? d.LS : d.U);
  const gptr<double> F64 = gp(adj ? d.LJ : d.F64);
  const gptr<float> F32 = gp(adj ? nullptr : d.F32);
  const int N = g.nx;
  const int nyq = (N & 1) ? -1 : N >> 1;  // Nyquist bin (even nx only)
  double2* a = sm;
  double2* b = sm + R * N;
  double2* tws = sm + 2 * R * N;  // twiddles staged in LDS
  for (int t = threadIdx.x; t < N; t += blockDim.x) tws[t] = gc2(d.twx)[t];
  const int s0 = 2 * pr, s1 = s0 + 1;
  const int g0 = adj ? s0 : kSrcG[s0], g1 = adj ? s1 : kSrcG[s1];
  const bool has1 = !adj || s1 < 3;
  for (int t = threadIdx.x; t < g.nxh * R; t += blockDim.x) {
    const int k = t / R, r = t - k * R;
    if (r >= nr) {  // past the last row: zero input, output not written
      a[r * N + k] = make_double2(0.0, 0.0);
      if (k > 0 && k != nyq) a[r * N + N - k] = make_double2(0.0, 0.0);
      continue;
    }
    const double kxs = 2.0 * M_PI * k / g.lx * ((k == nyq) ? 0.0 : 1.0);
    double2 X = U[((size_t)g0 * g.nxh + k) * g.ny + y0 + r];
    double2 Y = make_double2(0.0, 0.0);
    if (has1) Y = U[((size_t)g1 * g.nxh + k) * g.ny + y0 + r];
    if (!adj && kMulKx[s0]) X = mul_i(cscale(X, kxs));
    if (!adj && kMulKx[s1]) Y = mul_i(cscale(Y, kxs));
    if (k == 0 || k == nyq) {  // real-signal spectrum: these bins are real
      X.y = 0.0;
      Y.y = 0.0;
    }
    a[r * N + k] = cadd(X, mul_i(Y));
    if (k > 0 && k != nyq) a[r * N + N - k] = cadd(cconj(X), mul_i(cconj(Y)));
  }
  __syncthreads();
  const double2* res = fft_lds<true>(a, b, N, R, tws);
  const size_t plane = (size_t)g.nx * g.ny;
  for (int t = threadIdx.x; t < nr * N; t += blockDim.x) {
    const int r = t / N, x = t - r * N;
    const size_t o = (size_t)(y0 + r) * N + x;
    const double2 z = res[t];
    if (f64out || !F32) {
      F64[s0 * plane + o] = z.x;
      if (has1) F64[s1 * plane + o] = z.y;
    }
    if (F32) {  // node-major record: slots s0, s0 + 1 of node o
      F32[o * kFieldSlots + s0] = (float)z.x;
      F32[o * kFieldSlots + s0 + 1] = (float)z.y;
    }
  }
}

// history slot [nxh][ny] (internal) <-> [ny][nxh] (external)
__global__ void k_hist_transpose(const double2* __restrict__ src, double2* __restrict__ dst, int nfield,
                                 GridP g, int to_external) {
  const size_t plane = (size_t)g.nxh * g.ny;
  for (size_t t = blockIdx.x * (size_t)blockDim.x + threadIdx.x; t < plane * nfield;
       t += (size_t)gridDim.x * blockDim.x) {
    const size_t f = t / plane, r = t - f * plane;
    if (to_external) {  // r = ky*nxh + kx
      const size_t ky = r / g.nxh, kx = r - ky * g.nxh;
      dst[t] = src[f * plane + kx * g.ny + ky];
    } else {  // r = kx*ny + ky
      const size_t kx = r / g.ny, ky = r - kx * g.ny;
      dst[t] = src[f * plane + ky * g.nxh + kx];
    }
  }
}

// Diagnostics over the half spectrum (one block).  Sums of w |f|^2 with
// w = 1 on the kx = 0 and kx = nx/2 columns and 2 elsewhere (Parseval for the
// half spectrum of a real field).
template <int SCHEME>
__global__ void __launch_bounds__(1024) k_field_diag(const double2* __restrict__ H, GridP g, SchemeCoef sc,
                                                     HistSlots hs, double* __restrict__ out) {
  __shared__ double red[6][1024];
  const size_t plane = (size_t)g.nxh * g.ny;
  double acc[6] = {0, 0, 0, 0, 0, 0};  // gauge, gauge_t, gauge_d, gauss, rho+divE parts, energy
  double accr = 0, accd = 0;
  auto at = [&](int slot, size_t m) { return H[(size_t)slot * plane + m]; };
  for (size_t m = threadIdx.x; m < plane; m += blockDim.x) {
    const int kx = (int)(m / g.ny), ky = (int)(m - (size_t)kx * g.ny);
    const double kxs = kx_sym(kx, g), kys = ky_sym(ky, g);
    const double wgt = (kx == 0 || 2 * kx == g.nx) ? 1.0 : 2.0;
    auto divA = [&](int slot) {
      const double2 X = at(slot, m), Y = at(slot + 1, m);
      return mul_i(make_double2(kxs * X.x + kys * Y.x, kxs * X.y + kys * Y.y));
    };
    double2 gt, gd, rho, phi, E[3], A[3];
    if (SCHEME == PIC_SCHEME_BDF) {
      gt = make_double2(0, 0);
      double2 dA[3] = {{0, 0}, {0, 0}, {0, 0}};
      for (int j = 0; j <= sc.k; ++j) {
        gt = cadd(gt, cscale(at(hs.phi[j], m), sc.a[j] / (sc.c * sc.c * sc.dt)));
        for (int l = 0; l < 3; ++l) dA[l] = cadd(dA[l], cscale(at(hs.A[j] + l, m), sc.a[j] / sc.dt));
      }
      gd = divA(hs.A[0]);
      phi = at(hs.phi[0], m);
      rho = at(hs.rho[0], m);
      E[0] = csub(mul_i(cscale(phi, -kxs)), dA[0]);
      E[1] = csub(mul_i(cscale(phi, -kys)), dA[1]);
      E[2] = cscale(dA[2], -1.0);
      for (int l = 0; l < 3; ++l) A[l] = at(hs.A[0] + l, m);
    } else if (SCHEME == PIC_SCHEME_CDF2) {
      gt = cscale(csub(at(hs.phi[0], m), at(hs.phi[1], m)), 1.0 / (sc.c * sc.c * sc.dt));
      gd = divA(hs.A[0]);
      // Gauss in each form's levels: phi averaged over n+3/2 and n-1/2
      // (explicit: phi^{n+1/2}); rho averaged the same way (implicit) or
      // rho^{n+1/2} (semi-implicit, explicit)
      phi = sc.form == 2 ? at(hs.phi[1], m) : cscale(cadd(at(hs.phi[0], m), at(hs.phi[2], m)), 0.5);
      rho = sc.form == 0 ? cscale(cadd(at(hs.rho[0], m), at(hs.rho[2], m)), 0.5) : at(hs.rho[1], m);
      double2 dA[3];
      for (int l = 0; l < 3; ++l) {
        dA[l] = cscale(csub(at(hs.A[0] + l, m), at(hs.A[1] + l, m)), 1.0 / sc.dt);
        A[l] = cscale(cadd(at(hs.A[0] + l, m), at(hs.A[1] + l, m)), 0.5);
      }
      E[0] = csub(mul_i(cscale(phi, -kxs)), dA[0]);
      E[1] = csub(mul_i(cscale(phi, -kys)), dA[1]);
      E[2] = cscale(dA[2], -1.0);
    } else {
      double Rn = 0.0, Rn1 = 0.0;  // R^{s,n} = sum b_i (1 - c_i), R^{s,n+1} = sum b_i c_i
      for (int i = 0; i < sc.stages; ++i) {
        Rn += sc.dirkB[i] * (1 - sc.dirkC[i]);
        Rn1 += sc.dirkB[i] * sc.dirkC[i];
      }
      if (sc.substep) {  // stage-value gauge: v_phi + c^2 div A
        gt = at(hs.vphi, m);
        gd = cscale(divA(hs.A[0]), sc.c * sc.c);
      } else {
        gt = cscale(csub(at(hs.phi[0], m), at(hs.phi[1], m)), -1.0);
        gd = cscale(cadd(cscale(divA(hs.A[1]), Rn), cscale(divA(hs.A[0]), Rn1)), -sc.c * sc.c * sc.dt);
      }
      phi = at(hs.phi[0], m);
      rho = at(hs.rho[0], m);
      E[0] = csub(mul_i(cscale(phi, -kxs)), at(hs.vA, m));
      E[1] = csub(mul_i(cscale(phi, -kys)), at(hs.vA + 1, m));
      E[2] = cscale(at(hs.vA + 2, m), -1.0);
      for (int l = 0; l < 3; ++l) A[l] = at(hs.A[0] + l, m);
    }
    const double2 gsum = cadd(gt, gd);
    const double2 divE = mul_i(make_double2(kxs * E[0].x + kys * E[1].x, kxs * E[0].y + kys * E[1].y));
    const double2 rr = cscale(rho, 1.0 / sc.eps0);
    const double2 gauss = csub(divE, rr);
    const double2 Bx = mul_i(cscale(A[2], kys)), By = mul_i(cscale(A[2], -kxs));
    const double2 Bz = mul_i(make_double2(kxs * A[1].x - kys * A[0].x, kxs * A[1].y - kys * A[0].y));
    auto n2 = [](double2 z) { return z.x * z.x + z.y * z.y; };
    acc[0] += wgt * n2(gsum);
    acc[1] += wgt * n2(gt);
    acc[2] += wgt * n2(gd);
    acc[3] += wgt * n2(gauss);
    accr += wgt * n2(rr);
    accd += wgt * n2(divE);
    acc[5] += wgt * (sc.eps0 * (n2(E[0]) + n2(E[1]) + n2(E[2])) + (n2(Bx) + n2(By) + n2(Bz)) / sc.mu0);
    if (m == 0) acc[4] = rho.x;
  }
  // rho and divE norms share slot 4's neighbours: pack them into the reduction
  double vals[6] = {acc[0], acc[1], acc[2], acc[3], accr, accd};
  double e = acc[5], ch = acc[4];
  for (int i = 0; i < 6; ++i) red[i][threadIdx.x] = vals[i];
  __syncthreads();
  for (int s = blockDim.x / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s)
      for (int i = 0; i < 6; ++i) red[i][threadIdx.x] += red[i][threadIdx.x + s];
    __syncthreads();
  }
  double sums[6];
  for (int i = 0; i < 6; ++i) sums[i] = red[i][0];
  __syncthreads();
  red[0][threadIdx.x] = e;
  red[1][threadIdx.x] = ch;
  __syncthreads();
  for (int s = blockDim.x / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) {
      red[0][threadIdx.x] += red[0][threadIdx.x + s];
      red[1][threadIdx.x] += red[1][threadIdx.x + s];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const double norm = g.dx * g.dy / ((double)g.nx * g.ny);  // dx dy * (1/N) sum |f^|^2
    out[0] = sqrt(norm * sums[0]);
    out[1] = sqrt(norm * sums[1]) + sqrt(norm * sums[2]);
    out[2] = sqrt(norm * sums[3]);
    out[3] = sqrt(norm * sums[4]) + sqrt(norm * sums[5]);
    out[4] = red[1][0] * g.dx * g.dy;
    out[5] = 0.5 * norm * red[0][0];
  }
}

}  // namespace

// ---------------------------------------------------------------------------
// host side

void fft_make_twiddles(int n, double* h) {
  for (int t = 0; t < n; ++t) {
    const long double ang = 2.0L * 3.14159265358979323846264338327950288L * t / n;
    h[2 * t] = (double)cosl(ang);
    h[2 * t + 1] = (double)(-sinl(ang));
  }
}

// rows per block of the row kernels: at most 8, within the LDS budget, and
// small enough that one instance's transform has 256 blocks or more (the row
// kernels are latency-bound: more, shorter blocks finish sooner).  C2R keeps
// R nx <= 1024: its (2 R + 1) nx complex values of LDS then let three blocks
// share a CU at nx = 512 (two rows per block there: the solve 4 us faster
// than with four)
int rows_r2c_R(int nx, int ny) {
  int R = 8;
  while (R > 2 && (R > ny || R * nx > 4096)) R >>= 1;
  while (R > 2 && 3 * (ny / R) < 256) R >>= 1;
  return R;
}
int rows_c2r_R(int nx, int ny) {
  int R = 8;
  while (R > 1 && (R > ny || R * nx > 1024)) R >>= 1;
  while (R > 2 && 6 * (ny / R) < 256) R >>= 1;
  return R;
}
// work buffers plus the staged twiddles (n complex entries)
size_t rows_r2c_lds_bytes(int nx, int ny) { return (size_t)(rows_r2c_R(nx, ny) + 1) * nx * sizeof(double2); }
size_t rows_c2r_lds_bytes(int nx, int ny) { return (size_t)(2 * rows_c2r_R(nx, ny) + 1) * nx * sizeof(double2); }
// inverse batch size of the column kernel and its LDS bytes (<= 160 KiB)
int columns_nb(int ny) { return ny <= 256 ? 8 : (ny <= 512 ? 4 : 2); }
// k_adj_columns: accumulators 4 ny, work buffers max(6, 2 nb) ny (bounded here
// by max(8, 2 nb)), twiddles
size_t adj_columns_lds_bytes(int ny) {
  const int nb = columns_nb(ny);
  return (size_t)(4 + std::max(8, 2 * nb) + (ny <= 512 ? 1 : 0)) * ny * sizeof(double2);
}

hipError_t launch_rows_r2c(const InstDesc* D, int ninst, int nblocks, size_t lds, hipStream_t s, bool adj) {
  (void)hipFuncSetAttribute((const void*)k_rows_r2c, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  hipLaunchKernelGGL(k_rows_r2c, dim3(nblocks), dim3(256), lds, s, D, ninst, adj ? 1 : 0);
  return hipGetLastError();
}

template <int SCHEME, int K>
static hipError_t launch_columns_split_t(const InstDesc* D, int ninst, int nblocks, size_t lds, HistSlots hs,
                                         int max_ny, hipStream_t s) {
  (void)hipFuncSetAttribute((const void*)k_columns_split<SCHEME, K>, hipFuncAttributeMaxDynamicSharedMemorySize,
                            (int)lds);
  const int threads = max_ny > 256 * kColMaxModes ? 512 : 256;
  hipLaunchKernelGGL((k_columns_split<SCHEME, K>), dim3(nblocks), dim3(threads), lds, s, D, ninst, hs);
  return hipGetLastError();
}

int columns_parts(int) { return kColParts; }
// output column, work buffers (4 ny), twiddles (ny <= 512), stage columns
// (two per sub-stepped DIRK stage)
size_t columns_split_lds_bytes(int ny, int nstage) {
  return (size_t)(5 + (ny <= 512 ? 1 : 0) + 2 * nstage) * ny * sizeof(double2);
}

hipError_t launch_columns(int scheme, int bdf_order, const InstDesc* D, int ninst, int nblocks, size_t lds,
                          HistSlots hs, int max_ny, hipStream_t s) {
  if (scheme == PIC_SCHEME_CDF2) return launch_columns_split_t<PIC_SCHEME_CDF2, 0>(D, ninst, nblocks, lds, hs, max_ny, s);
  if (scheme == PIC_SCHEME_DIRK2) return launch_columns_split_t<PIC_SCHEME_DIRK2, 0>(D, ninst, nblocks, lds, hs, max_ny, s);
  switch (bdf_order) {
    case 1: return launch_columns_split_t<PIC_SCHEME_BDF, 1>(D, ninst, nblocks, lds, hs, max_ny, s);
    case 2: return launch_columns_split_t<PIC_SCHEME_BDF, 2>(D, ninst, nblocks, lds, hs, max_ny, s);
    case 3: return launch_columns_split_t<PIC_SCHEME_BDF, 3>(D, ninst, nblocks, lds, hs, max_ny, s);
    case 4: return launch_columns_split_t<PIC_SCHEME_BDF, 4>(D, ninst, nblocks, lds, hs, max_ny, s);
    case 5: return launch_columns_split_t<PIC_SCHEME_BDF, 5>(D, ninst, nblocks, lds, hs, max_ny, s);
    default: return launch_columns_split_t<PIC_SCHEME_BDF, 6>(D, ninst, nblocks, lds, hs, max_ny, s);
  }
}

__global__ void k_j_export(const long long* __restrict__ src, double* __restrict__ dst, size_t n, double unscale) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
    dst[i] = (double)src[i] * unscale;
}

hipError_t launch_j_export(const long long* src, double* dst, size_t n, double unscale, hipStream_t s) {
  const int blocks = (int)std::min<size_t>(4096, (n + 255) / 256);
  if (n) hipLaunchKernelGGL(k_j_export, dim3(blocks), dim3(256), 0, s, src, dst, n, unscale);
  return hipGetLastError();
}

hipError_t launch_rows_c2r(const InstDesc* D, int ninst, int nblocks, size_t lds, hipStream_t s, bool adj,
                           bool f64out) {
  (void)hipFuncSetAttribute((const void*)k_rows_c2r, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  hipLaunchKernelGGL(k_rows_c2r, dim3(nblocks), dim3(256), lds, s, D, ninst, adj ? 1 : 0, f64out ? 1 : 0);
  return hipGetLastError();
}

hipError_t launch_hist_transpose(const double2* src, double2* dst, int nfield, GridP g, bool to_external,
                                 hipStream_t s) {
  const size_t n = (size_t)g.nxh * g.ny * nfield;
  const int blocks = (int)std::min<size_t>((n + 255) / 256, 4096);
  hipLaunchKernelGGL(k_hist_transpose, dim3(blocks), dim3(256), 0, s, src, dst, nfield, g,
                     to_external ? 1 : 0);
  return hipGetLastError();
}

hipError_t launch_field_diag(const double2* H, GridP g, SchemeCoef sc, HistSlots hs, double* out,
                             hipStream_t s) {
  if (sc.scheme == PIC_SCHEME_BDF)
    hipLaunchKernelGGL(k_field_diag<PIC_SCHEME_BDF>, dim3(1), dim3(1024), 0, s, H, g, sc, hs, out);
  else if (sc.scheme == PIC_SCHEME_CDF2)
    hipLaunchKernelGGL(k_field_diag<PIC_SCHEME_CDF2>, dim3(1), dim3(1024), 0, s, H, g, sc, hs, out);
  else
    hipLaunchKernelGGL(k_field_diag<PIC_SCHEME_DIRK2>, dim3(1), dim3(1024), 0, s, H, g, sc, hs, out);
  return hipGetLastError();
}

}  // namespace pic
