/*
 * pic.h -- C ABI of libpic: the per-step particle-mesh hot path of the
 * gauge-conserving PIC method with generalized momentum (arXiv 2410.18414),
 * on a periodic 2-D grid, 2D3V, one mobile species of macro-particles.
 *
 * One step is Algorithm 1 (Sec. 4.2):
 *   deposit_current  x^{n+1} = x^n + v^n dt (periodic wrap); J^{n+1} by
 *                    tensor-product B-spline deposition of q v^n at x^{n+1}
 *                    (Sec. 2.2 PIC current density; Sec. 4.1).
 *   field_solve      FFT of J; rho from the stepper's continuity equation;
 *                    phi and A by BDF-k (Sec. 3.2), implicit CDF-2 (Sec. 3.1)
 *                    or DIRK-2 (Sec. 3.3), each modified-Helmholtz operator
 *                    L = I - Laplacian/alpha^2 inverted mode by mode in Fourier
 *                    space; spectral gradients of phi~ and A on the mesh
 *                    (Sec. 4.1: derivatives must be spectral).
 *   gather_push      interpolate the mesh fields at x^{n+1} with the same
 *                    spline; IAEM push (Sec. 4.1): v* = 2v^n - v^{n-1},
 *                    P^{n+1} = P^n + q(-grad phi~ + (grad A).v*) dt,
 *                    v^{n+1} = c^2 (P - qA)/sqrt(c^2 |P - qA|^2 + (m c^2)^2);
 *                    shift the history.
 *   step             nsteps x (deposit_current, field_solve, gather_push),
 *                    with the gather/push of step n fused with the deposit of
 *                    step n+1 (same results).  Its launches repeat with a
 *                    period of a few steps; step() captures one period into a
 *                    HIP graph (on an internal stream) and replays it on the
 *                    context's stream.
 *
 * Conventions
 *   - Pointers are DEVICE pointers unless marked [host].  Work is enqueued
 *     asynchronously on the HIP stream given to pic_create; results are valid
 *     once that stream has synchronised.  Calls returning data to [host]
 *     memory synchronise the stream themselves.
 *   - Mesh nodes sit at (i dx, j dy), i < nx, j < ny; real mesh arrays are
 *     row-major [ny][nx] float64 (x fastest).  Spectral arrays are the
 *     half spectrum [ny][nx/2+1] of complex128 (interleaved re, im), forward
 *     transform unnormalised with exp(-i k.x).
 *   - Particle arrays passed in or out are float64 SoA blocks of length n.
 *   - The caller allocates the workspace (pic_workspace_bytes) and owns it
 *     and every buffer it passes; the library allocates no device memory.
 *   - Errors: arguments are validated before anything is enqueued; on error
 *     nothing is enqueued, the context is unchanged, and pic_last_error()
 *     describes the failure.  No call aborts the process.
 *   - A context is not thread-safe.
 */
#ifndef PIC_H
#define PIC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define PIC_ABI_VERSION 1

typedef struct pic_ctx_s* pic_ctx_t;

typedef enum {
  PIC_OK = 0,
  PIC_ERR_INVALID_ARG = 1, /* a pointer, size or parameter is invalid          */
  PIC_ERR_UNSUPPORTED = 2, /* a valid parameter the library does not implement */
  PIC_ERR_WORKSPACE = 3,   /* workspace too small or misaligned (256 B)        */
  PIC_ERR_HIP = 4,         /* a HIP runtime call or launch failed              */
  PIC_ERR_STATE = 5,       /* call out of order (see the phase rules below)    */
  PIC_ERR_NONFINITE = 6    /* pic_diagnostics found a NaN/Inf particle value   */
} pic_status_t;

/* PIC_SCHEME_CDF2 is the implicit centred-difference form of Sec. 3.1 (sources
 * averaged over n+1 and n-1); PIC_SCHEME_CDF2_SEMI and PIC_SCHEME_CDF2_EXPLICIT
 * are its semi-implicit and explicit forms (sources rho^{n+1/2}, J^n; the
 * Laplacian averaged over n+1 and n-1, or at level n -- the explicit wave
 * update is stable for c dt |k| <= 2 on every mode).  All three take
 * rho^{n+3/2} from the staggered continuity equation with J^{n+1} and push
 * with phi~ = (phi^{n+3/2} + phi^{n+1/2})/2; their history layout is the same. */
typedef enum {
  PIC_SCHEME_BDF = 0,
  PIC_SCHEME_CDF2 = 1,
  PIC_SCHEME_DIRK2 = 2,
  PIC_SCHEME_CDF2_SEMI = 3,
  PIC_SCHEME_CDF2_EXPLICIT = 4,
  /* three-stage DIRK (Sec. 3.3, s = 3): implicit-midpoint substeps of lengths
   * b_i dt composed in sequence (a_ij = b_j for j < i, a_ii = b_i/2), with the
   * fourth-order weights b_1 = b_3 = 1/(2 - 2^{1/3}), b_2 = 1 - 2 b_1; the
   * composition with b = (1/2, 1/2) is DIRK-2's tableau.  Same history layout
   * as PIC_SCHEME_DIRK2. */
  PIC_SCHEME_DIRK3 = 5
} pic_scheme_t;
typedef enum { PIC_F32 = 0, PIC_F64 = 1 } pic_dtype_t;

/* flags */
#define PIC_FLAG_NO_SORT 1u      /* never reorder particles by tile            */
#define PIC_FLAG_UNFUSED_STEP 2u /* step() runs the three calls separately     */
#define PIC_FLAG_NO_GRAPH 4u     /* step() never replays a captured HIP graph    */
#define PIC_FLAG_ADJOINT 8u      /* reserve the adjoint buffers (step_adjoint)   */
/* The paper's naive comparison (Sec. 5.1, the "naive update" of the Weibel
 * figures): rho^{n+1} is mapped to the mesh from the particles at x^{n+1} with
 * the same spline as J (the PIC charge density of Sec. 2.2), plus an immobile
 * ion background equal to minus the electron charge of init_particles (so
 * rho^0 = 0), and replaces the continuity update.  BDF-k and DIRK-2 only
 * (CDF-2 needs rho at half levels): PIC_ERR_UNSUPPORTED otherwise, and with
 * PIC_FLAG_ADJOINT.  The particle passes are the untiled ones (global atomics). */
#define PIC_FLAG_NAIVE_RHO 16u
/* J^{n+1} carries the extrapolated velocity v* = 2 v^n - v^{n-1} of the push
 * (Sec. 4.2, the alternative the paper allows for the current) instead of v^n;
 * positions still move with v^n.  rho follows from continuity with that J, so
 * the gauge property is unchanged.  Every scheme and spline; not with
 * PIC_FLAG_ADJOINT (PIC_ERR_UNSUPPORTED). */
#define PIC_FLAG_JVSTAR 32u
/* DIRK stage currents by particle sub-stepping (the alternative to linear
 * interpolation named with the DIRK continuity update of Algorithm 1): stage i
 * deposits J^(i) from the particles advanced by the IAEM position update over
 * c_i dt (x^n + c_i dt v^n, weighted by q v^n, or q v* with PIC_FLAG_JVSTAR),
 * one deposit pass per stage.  The stage charge densities are the RK stage
 * values of the continuity equation, rho^(i) = rho^n - dt sum_{j<=i} a_ij
 * div J^(i), so v_phi + c^2 div A = 0 and Gauss's law (E = -grad phi - v_A)
 * hold to round-off; pic_diagnostics reports that gauge form.  The DIRK J
 * history level holds sum_i b_i J^(i).  DIRK-2 and DIRK-3 only; not with
 * PIC_FLAG_NAIVE_RHO or PIC_FLAG_ADJOINT (PIC_ERR_UNSUPPORTED).  step() runs
 * the gather/push and the stage deposits as separate passes. */
#define PIC_FLAG_DIRK_SUBSTEP 64u
/* Deterministic deposit: J is accumulated in 64-bit integers at a fixed
 * power-of-two scale per instance (the LDS windows and their flush alike), so
 * every sum is exact and independent of the order particles or workgroups
 * arrive in; runs repeat bit for bit (and a resumed run equals the
 * uninterrupted one).  The quantisation is one rounding per contribution at
 * the fixed scale (float32 particles: the same scale the default mode uses
 * for full chunks; float64: below 2^-40 of the largest contribution).  Sorted
 * passes only: PIC_ERR_UNSUPPORTED with PIC_FLAG_NO_SORT, PIC_FLAG_NAIVE_RHO
 * or PIC_FLAG_ADJOINT. */
#define PIC_FLAG_DETERMINISTIC 128u

typedef struct {                /* [host] */
  int32_t abi_version;          /* == PIC_ABI_VERSION                                    */
  int32_t nx, ny;               /* mesh nodes per axis, 8 .. 1024 (any integer: mixed-
                                   radix FFTs; powers of two take the compiled tile
                                   geometries and are required by PIC_FLAG_ADJOINT)     */
  int32_t spline_degree;        /* 1 (linear), 2 (quadratic, the paper's), 3 (cubic),
                                   4, 5 (quartic, quintic; not with the adjoint)         */
  double lx, ly;                /* periodic box [0,lx) x [0,ly)                          */
  int32_t scheme;               /* pic_scheme_t                                          */
  int32_t bdf_order;            /* BDF-k order 1..6 (Sec. 3.2), used when scheme == BDF  */
  int32_t particle_dtype;       /* pic_dtype_t of particle state and gather; mesh FFT and
                                   spectral history are float64 in both cases           */
  int32_t sort_interval;        /* position updates between re-sorts; 0 = from the
                                   particles init_particles loads: slack / (max(|v_x|,
                                   |v_y|) dt / min(dx, dy)), kept between the speed-of-
                                   light interval and three times it (a particle that leaves
                                   its window takes the global path: results never
                                   depend on the interval)                              */
  double dt;                    /* time step                                             */
  double c, eps0, mu0;          /* |c^2 eps0 mu0 - 1| <= 1e-12 required (Sec. 2.1)      */
  double q, m;                  /* macro-particle charge and mass                        */
  int64_t max_particles;        /* capacity, >= 1                                        */
  uint32_t flags;               /* PIC_FLAG_*                                            */
  int32_t tile_cells;           /* tile edge in cells for the sorted passes (power of two,
                                   4..64, at most nx and ny); 0 = default (16, or the
                                   largest power of two not above nx and ny); a side
                                   that is no multiple of it ends in a partial tile     */
  int32_t chunk;                /* particles per workgroup of the sorted passes
                                   (64..65536); 0 = default: the largest of 512, 1024,
                                   2048, 4096 leaving >= 8192 chunks at max_particles    */
  int32_t slack;                /* cells a particle may drift from its tile and still use
                                   the tile's LDS window (1..8); 0 = default (3); at
                                   most min(nx, ny) - 2 when a side is no power of two */
  int32_t reserved[4];          /* must be zero                                          */
} pic_config_t;

/* Workspace bytes pic_create needs for cfg (0 if cfg is invalid). */
size_t pic_workspace_bytes(const pic_config_t* cfg);

/* Create a context.  workspace: device buffer of ws_bytes >= pic_workspace_bytes,
 * 256-byte aligned, owned by the caller and untouched by it until pic_destroy.
 * hip_stream: hipStream_t to enqueue on (NULL = default stream).  Zero-fills
 * the field history (cold start: all levels n <= 0 vanish). */
pic_status_t pic_create(const pic_config_t* cfg, void* workspace, size_t ws_bytes,
                        void* hip_stream, pic_ctx_t* out);
void pic_destroy(pic_ctx_t ctx);

/* Message of the last failed call on ctx; with ctx == NULL, of the last failed
 * pic_create / pic_workspace_bytes on this thread. */
const char* pic_last_error(pic_ctx_t ctx);

/* Load n particles: x[n], y[n] positions (wrapped into the box) and P[3n]
 * generalized momenta as blocks Px, Py, Pz (float64, device).  With the cold
 * start A^0 = 0, so v^0 = c^2 P/sqrt(c^2 |P|^2 + (m c^2)^2) (Sec. 2.2); the
 * Taylor start of Algorithm 1 gives v^{-1} = v^0 because the t = 0 force
 * vanishes.  Resets the step counter and the field history.  Phase -> READY. */
pic_status_t init_particles(pic_ctx_t ctx, int64_t n, const double* x, const double* y,
                            const double* P);

/* READY -> DEPOSITED.  Position update and current deposition (Algorithm 1,
 * first two steps). */
pic_status_t deposit_current(pic_ctx_t ctx);
/* DEPOSITED -> SOLVED.  Continuity, field update, spectral gradients
 * (Algorithm 1, steps three to five). */
pic_status_t field_solve(pic_ctx_t ctx);
/* SOLVED -> READY.  Gather, IAEM push, history shift (Algorithm 1, remaining
 * steps). */
pic_status_t gather_push(pic_ctx_t ctx);
/* READY -> READY.  nsteps >= 0 complete steps. */
pic_status_t step(pic_ctx_t ctx, int32_t nsteps);
/* Steps in one replayed graph period (0: step() launches every kernel
 * itself -- PIC_FLAG_NO_GRAPH, kernel timing on, or unsorted passes).  The
 * first step() call of more than this many steps captures and instantiates
 * the graph, a one-time host cost; later calls replay it, after at most
 * period - 1 directly launched steps that bring the launch state back to the
 * captured one. */
int32_t pic_graph_period(pic_ctx_t ctx);

/* Particle state in the ORIGINAL particle order, float64 device out[11 n]:
 * blocks x, y, Px, Py, Pz, vx^n, vy^n, vz^n, vx^{n-1}, vy^{n-1}, vz^{n-1}. */
pic_status_t pic_get_particles(pic_ctx_t ctx, double* out);
/* Replace the particle state (same layout, original order) in phase READY or
 * SOLVED; phase -> READY.  Values are rounded to the particle dtype; positions
 * are wrapped. */
pic_status_t pic_set_particles(pic_ctx_t ctx, const double* in);

/* Saved states: the complete state of a context in phase READY or SOLVED
 * (every instance's particles in their current sorted order with their
 * original indices, the tile metadata of the last sort, the spectral history
 * ring, the step, ring and sort counters, and in phase SOLVED the mesh fields
 * of the last solve), in a caller-owned DEVICE buffer of
 * pic_state_bytes(ctx) bytes, 256-byte aligned.  pic_save_state enqueues
 * device-to-device copies (no synchronisation, no allocation); pic_load_state
 * restores a state saved by a context of the same configuration (it reads
 * the buffer's header, synchronising the stream), after
 * which the context steps exactly as it would have from the saved point --
 * no conversion to float64 and no re-sort, unlike pic_get/set_particles and
 * pic_get/set_history.  pic_load_state accepts any phase (it replaces the
 * whole state and leaves the saved phase, READY or SOLVED); pic_save_state
 * returns PIC_ERR_STATE in phases EMPTY and DEPOSITED.  The layout is private
 * to the library version:
 * PIC_ERR_INVALID_ARG for a buffer from another configuration or not 256-byte
 * aligned. */
size_t pic_state_bytes(pic_ctx_t ctx);
pic_status_t pic_save_state(pic_ctx_t ctx, void* dst);
pic_status_t pic_load_state(pic_ctx_t ctx, const void* src);

/* The same without the header read: pic_save_state_h also writes the state's
 * header, pic_state_header_words(ctx) int64 words, to [host] header (NULL:
 * not written); pic_load_state_h takes the header from [host] header instead
 * of reading it from src, so it neither synchronises the stream nor waits for
 * the save to finish (for loops that save and reload many states, e.g. an
 * adjoint sweep).  header must be the one pic_save_state_h wrote for src, and
 * src unchanged since; it holds pic_state_header_words(ctx) words of the
 * loading context (a header of another instance count would be read past its
 * end); the same validation of the header words applies.
 * header NULL: pic_load_state. */
int32_t pic_state_header_words(pic_ctx_t ctx);
pic_status_t pic_save_state_h(pic_ctx_t ctx, void* dst, int64_t* header);
pic_status_t pic_load_state_h(pic_ctx_t ctx, const void* src, const int64_t* header);

/* Real mesh fields, float64 device dst:
 *   PIC_FIELD_J      [3][ny][nx]  J^{n+1}; valid in phase DEPOSITED
 *                    (PIC_FLAG_DIRK_SUBSTEP: [3 stages][ny][nx], stage i at
 *                    planes 3i .. 3i+2)
 *   PIC_FIELD_MESH  [12][ny][nx]  the gathered fields, valid in phase SOLVED:
 *        dphi/dx, dphi/dy, Ax, Ay, Az, dAx/dx, dAy/dx, dAz/dx,
 *        dAx/dy, dAy/dy, dAz/dy, phi~   (phi~ = phi^{n+1}; CDF-2: the mean
 *        of phi^{n+3/2} and phi^{n+1/2}, Sec. 4.1) */
#define PIC_FIELD_J 0
#define PIC_FIELD_MESH 1
pic_status_t pic_get_field(pic_ctx_t ctx, int32_t which, double* dst);

/* Spectral field history, pic_history_fields(cfg) complex half spectra
 * [ny][nx/2+1], newest level first within each group:
 *   BDF-k : rho (k levels), phi (2k), A (2k levels x 3 components)
 *   CDF-2 : rho^{n+1/2..n-3/2} (3), phi (3), A^{n..n-1} (2 x 3), J^{n..n-1} (2 x 3)
 *   DIRK-2: rho (2), phi (2), v_phi (1), A (2 x 3), v_A (3), J^n (3)
 *           (DIRK-3 the same; with PIC_FLAG_DIRK_SUBSTEP the J level is
 *           sum_i b_i J^(i) of the last step)
 * (v_phi, v_A: the time derivatives the DIRK first-order system carries.) */
int32_t pic_history_fields(const pic_config_t* cfg);
pic_status_t pic_get_history(pic_ctx_t ctx, double* dst);
pic_status_t pic_set_history(pic_ctx_t ctx, const double* src);

/* Diagnostics of the newest level (untimed, synchronises the stream).
 * [host] out[PIC_DIAG_COUNT]:
 *   0 gauge residual L2   1 gauge scale   2 Gauss residual L2   3 Gauss scale
 *   4 total charge        5 field energy  6 particle kinetic energy
 *   7 non-finite particle values (count)
 * Residuals as defined per stepper in Sec. 3 (epsilon_1 and Gauss's law);
 * L2 = sqrt(dx dy sum f^2) by Parseval.  Returns PIC_ERR_NONFINITE when
 * out[7] > 0 (the values are still written). */
#define PIC_DIAG_COUNT 8
pic_status_t pic_diagnostics(pic_ctx_t ctx, double* out);

/* General s-stage DIRK (Sec. 3.3: the stage equations, the continuity update
 * and the gauge theorem are stated for any diagonally implicit tableau).
 * Replaces the tableau of a PIC_SCHEME_DIRK2 / PIC_SCHEME_DIRK3 context (every
 * instance of an ensemble) by [host] A[stages*stages] (row-major, lower
 * triangular, positive diagonal: each stage solves one modified-Helmholtz
 * problem with alpha_i = 1/(dt a_ii c)), b[stages] (summing to one) and
 * c[stages] (the row sums of A; stage currents interpolate J^n and J^{n+1} at
 * c_i, or are deposited at x^n + c_i dt v^n with PIC_FLAG_DIRK_SUBSTEP).
 * stages must be the scheme's: 2 for PIC_SCHEME_DIRK2, 3 for
 * PIC_SCHEME_DIRK3.  Phase READY or before particles are loaded; the next
 * steps use the new tableau (the history layout does not change).
 * PIC_ERR_UNSUPPORTED for other schemes, PIC_ERR_INVALID_ARG for a tableau
 * outside these rules. */
pic_status_t pic_set_dirk_tableau(pic_ctx_t ctx, int32_t stages, const double* A, const double* b,
                                  const double* c);

/* Diagnostics of every instance, for callers that cannot allocate device
 * memory or synchronise (code under HIP graph capture, serving loops): the
 * values of pic_diagnostics for each instance i of the context (the selected
 * one alone for a plain context) are written to the DEVICE array
 * out[i * PIC_DIAG_COUNT + k], in the pic_diagnostics order, by kernels
 * enqueued on the context's stream; nothing is synchronised, no device memory
 * is allocated and no host buffer is touched (results are valid once the
 * stream has synchronised; a non-finite particle shows in out[i*8 + 7], and
 * the call itself returns PIC_OK).  The reduction partials live in a fixed
 * scratch array of the library, PIC_DIAG_ALL_MAX instances x 528 doubles
 * (270 KB), one copy per GPU the library runs on, held until the process
 * ends; contexts with more instances get PIC_ERR_INVALID_ARG.  Every call on
 * one GPU shares that GPU's scratch: calls that overlap in time on one GPU
 * (from two streams or two host threads) race and may return each other's
 * values; calls ordered on one stream do not. */
#define PIC_DIAG_ALL_MAX 64
pic_status_t pic_diagnostics_all(pic_ctx_t ctx, double* out);

/* ---- Ensembles (batched instances) ----------------------------------------
 * A context may hold ninst independent instances of the method: an ensemble
 * of uneven workloads (different grids, particle counts, time steps).  They must share scheme, bdf_order, particle_dtype, spline_degree,
 * flags and c, eps0, mu0.  Every hot-path kernel then covers all instances in
 * one launch per phase (a flattened grid), and the instances advance in
 * lockstep: deposit_current, field_solve, gather_push, step and step_batched
 * act on all of them.  init_particles, pic_get/set_particles, pic_get_field,
 * pic_get/set_history and pic_diagnostics act on the instance chosen with
 * pic_select_instance (0 after creation).  In an ensemble, every instance is
 * loaded with init_particles before the first step. */
size_t pic_batch_workspace_bytes(const pic_config_t* cfgs, int32_t ninst);
pic_status_t pic_batch_create(const pic_config_t* cfgs, int32_t ninst, void* workspace, size_t ws_bytes,
                              void* hip_stream, pic_ctx_t* out);
int32_t pic_instance_count(pic_ctx_t ctx);
pic_status_t pic_select_instance(pic_ctx_t ctx, int32_t index);
/* nsteps complete steps of every instance (the same as step()). */
pic_status_t step_batched(pic_ctx_t ctx, int32_t nsteps);

/* ---- Discrete adjoint (reverse mode) -------------------------------------
 * The exact transpose of one step's Jacobian, for gradients of a function of
 * the final state with respect to the initial particles.  Float64 particles,
 * the BDF-k stepper (Sec. 3.2), single-instance contexts created with
 * PIC_FLAG_ADJOINT (else PIC_ERR_UNSUPPORTED).  A state S^n is the particle
 * arrays of pic_get_particles plus the history of pic_get_history.
 *
 * Adjoint state (device float64, caller-owned, updated in place):
 *   lam       [11][n]  d(loss)/d(particle state), the pic_get_particles layout
 *                      and original particle order
 *   lam_hist  [pic_history_fields][ny][nx/2+1] complex (re, im pairs):
 *                      d(loss)/d(history), the pic_get_history layout; the
 *                      adjoint of a complex value z is dL/dRe z + i dL/dIm z.
 *
 * adjoint_seed_energy: phase READY.  lam_hist = scale * dW/d(history) for the
 * field energy W of the newest level (pic_diagnostics out[5]: E from the
 * BDF-k time derivative of A, Sec. 2.2 and 3.2).  The particle adjoint of W is
 * zero (the caller clears lam).
 *
 * step_adjoint: phase READY with the context holding S^n, or phase SOLVED
 * with S^n advanced by deposit_current + field_solve (a state saved there by
 * pic_save_state, or those two calls).  In phase READY it first recomputes
 * the position update, deposit and field solve of step n -> n+1 (as
 * deposit_current + field_solve, but without re-sorting particles whose
 * order comes from a sort: a particle that has drifted past its tile's
 * window takes the global path, and the held adjoint keeps its order).
 * Phase -> SOLVED afterwards, marked as used: a second step_adjoint before
 * another state is loaded (pic_load_state, or pic_set_particles and
 * pic_set_history) or solved returns PIC_ERR_STATE.  It maps
 * (lam, lam_hist) = lambda^{n+1} to lambda^n =
 * (dS^{n+1}/dS^n)^T lambda^{n+1}: the push and gather adjoint (a scatter onto
 * the 11 gathered mesh fields; spline derivative weights for the position),
 * the field-solve adjoint (conjugate transforms and the transposed per-mode
 * BDF recurrence) and the deposit adjoint (a gather of d/dJ with spline and
 * derivative weights).  Wrap-around of positions counts as the identity.
 * lam NULL: the particle adjoint is the one the context holds (below) and
 * stays there, so a sweep of many steps exchanges it only at its ends.
 *
 * The held particle adjoint: the context keeps lam in the order of its
 * particle slots, so the adjoint passes read and write it with contiguous
 * accesses; it is permuted only when a sort changes the order.  The context
 * tags each slot order when it is made (sort, init_particles, set_particles;
 * a saved state keeps its tag); when the loaded particles carry another tag
 * than the order the adjoint follows, a device-side check (no host
 * synchronisation) compares the orders and permutes if they differ.
 * pic_adjoint_set_particles: lam [11][n] in original order (NULL: zero) into
 * the context, for the particles loaded now.  pic_adjoint_get_particles: the
 * held adjoint back out in original order (PIC_ERR_STATE if none is held for
 * the loaded particle count).  step_adjoint with a non-NULL lam is
 * set_particles, the NULL form, get_particles.
 *
 * adjoint_initial: any loaded phase.  Maps the adjoint of S^0 to the adjoint of
 * the init_particles inputs, P0 [3n] as given to init_particles (original
 * order): lam[Px..Pz] += (dv^0/dP)^T (lam[v^n] + lam[v^{n-1}]) (both start at
 * v^0), then the velocity blocks of lam are cleared; lam[x], lam[y] are
 * already d/dx0, d/dy0. */
pic_status_t adjoint_seed_energy(pic_ctx_t ctx, double scale, double* lam_hist);
pic_status_t step_adjoint(pic_ctx_t ctx, double* lam, double* lam_hist);
pic_status_t pic_adjoint_set_particles(pic_ctx_t ctx, const double* lam);
pic_status_t pic_adjoint_get_particles(pic_ctx_t ctx, double* lam);
pic_status_t adjoint_initial(pic_ctx_t ctx, const double* P0, double* lam);

/* Kernel timing with HIP events recorded on the context's stream around each
 * launch group (for roofline reporting; adds an event pair per launch).
 * Classes: 0 deposit (position update + deposit), 1 field solve (R2C rows,
 * column update, C2R rows), 2 gather + push, 3 fused gather/push/deposit,
 * 4 tile sort (count, scan, scatter).
 * pic_kernel_timing synchronises the stream, writes [host] out[2*PIC_KCLASS_COUNT]
 * = {total ms, launches} per class, and resets the counters. */
#define PIC_KCLASS_COUNT 5
pic_status_t pic_set_kernel_timing(pic_ctx_t ctx, int32_t enable);
pic_status_t pic_kernel_timing(pic_ctx_t ctx, double* out);

#ifdef __cplusplus
}
#endif
#endif /* PIC_H */
