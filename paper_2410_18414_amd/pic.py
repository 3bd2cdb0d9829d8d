"""Thin ctypes binding of libpic (include/pic.h): argument marshalling only.

Every step of the PIC path runs in libpic's HIP kernels; PyTorch supplies the
device memory (workspace, particle inputs/outputs) and the HIP stream.  There
is no fallback: if libpic.so is missing, :func:`load` raises.

    ctx = Context(Config(nx=128, ny=128, lx=12.8, ly=12.8, ...), max_particles=n)
    init_particles(ctx, x, y, P)      # float64 CUDA tensors
    step(ctx, 10)
    parts = get_particles(ctx)        # [11, n] float64, original order
"""

import ctypes
import os

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libpic.so")

PIC_ABI_VERSION = 1
SCHEMES = {"bdf": 0, "cdf2": 1, "dirk2": 2, "cdf2_semi": 3, "cdf2_explicit": 4, "dirk3": 5}
DTYPES = {"f32": 0, "f64": 1}
FLAG_NO_SORT = 1
FLAG_UNFUSED_STEP = 2
FLAG_NO_GRAPH = 4
FLAG_ADJOINT = 8
FLAG_NAIVE_RHO = 16   # rho deposited with the spline instead of continuity (the paper's naive update)
FLAG_JVSTAR = 32      # J carries v* = 2 v^n - v^{n-1} instead of v^n
FLAG_DIRK_SUBSTEP = 64  # DIRK stage currents from particles sub-stepped to each stage time
FLAG_DETERMINISTIC = 128  # J summed in int64 at a fixed scale: runs repeat bit for bit
FIELD_J = 0
FIELD_MESH = 1
DIAG_ALL_MAX = 64  # instances pic_diagnostics_all covers (its scratch size)
DIAG_NAMES = ("gauge_l2", "gauge_scale", "gauss_l2", "gauss_scale", "charge", "energy",
              "kinetic", "nonfinite")
STATUS = {0: "PIC_OK", 1: "PIC_ERR_INVALID_ARG", 2: "PIC_ERR_UNSUPPORTED", 3: "PIC_ERR_WORKSPACE",
          4: "PIC_ERR_HIP", 5: "PIC_ERR_STATE", 6: "PIC_ERR_NONFINITE"}

# every entry point pic.h declares (checked by the CPU test suite)
EXPORTS = ("pic_workspace_bytes", "pic_create", "pic_destroy", "pic_last_error",
           "init_particles", "deposit_current", "field_solve", "gather_push", "step",
           "pic_get_particles", "pic_set_particles", "pic_get_field", "pic_history_fields",
           "pic_get_history", "pic_set_history", "pic_diagnostics", "pic_set_kernel_timing",
           "pic_kernel_timing", "pic_batch_workspace_bytes", "pic_batch_create",
           "pic_instance_count", "pic_select_instance", "step_batched", "adjoint_seed_energy",
           "step_adjoint", "adjoint_initial", "pic_graph_period", "pic_diagnostics_all",
           "pic_set_dirk_tableau", "pic_state_bytes", "pic_save_state", "pic_load_state",
           "pic_adjoint_set_particles", "pic_adjoint_get_particles", "pic_state_header_words",
           "pic_save_state_h", "pic_load_state_h")
KCLASSES = ("deposit", "field_solve", "gather_push", "fused", "sort")


class PicError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__("%s: %s" % (STATUS.get(status, status), msg))
        self.status = status


class ConfigStruct(ctypes.Structure):
    _fields_ = [("abi_version", ctypes.c_int32), ("nx", ctypes.c_int32), ("ny", ctypes.c_int32),
                ("spline_degree", ctypes.c_int32), ("lx", ctypes.c_double), ("ly", ctypes.c_double),
                ("scheme", ctypes.c_int32), ("bdf_order", ctypes.c_int32),
                ("particle_dtype", ctypes.c_int32), ("sort_interval", ctypes.c_int32),
                ("dt", ctypes.c_double), ("c", ctypes.c_double), ("eps0", ctypes.c_double),
                ("mu0", ctypes.c_double), ("q", ctypes.c_double), ("m", ctypes.c_double),
                ("max_particles", ctypes.c_int64), ("flags", ctypes.c_uint32),
                ("tile_cells", ctypes.c_int32), ("chunk", ctypes.c_int32), ("slack", ctypes.c_int32),
                ("reserved", ctypes.c_int32 * 4)]


_lib = None


def load():
    """Load libpic.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError("libpic.so not built: run python -m paper_2410_18414_amd.build")
    lib = ctypes.CDLL(LIB_PATH)
    P, I32, I64, SZ, D = (ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_size_t,
                          ctypes.c_double)
    cfgp = ctypes.POINTER(ConfigStruct)
    sig = {
        "pic_workspace_bytes": (SZ, [cfgp]),
        "pic_create": (I32, [cfgp, P, SZ, P, ctypes.POINTER(P)]),
        "pic_destroy": (None, [P]),
        "pic_last_error": (ctypes.c_char_p, [P]),
        "init_particles": (I32, [P, I64, P, P, P]),
        "deposit_current": (I32, [P]),
        "field_solve": (I32, [P]),
        "gather_push": (I32, [P]),
        "step": (I32, [P, I32]),
        "pic_get_particles": (I32, [P, P]),
        "pic_set_particles": (I32, [P, P]),
        "pic_get_field": (I32, [P, I32, P]),
        "pic_history_fields": (I32, [cfgp]),
        "pic_get_history": (I32, [P, P]),
        "pic_set_history": (I32, [P, P]),
        "pic_diagnostics": (I32, [P, ctypes.POINTER(D)]),
        "pic_diagnostics_all": (I32, [P, P]),
        "pic_set_dirk_tableau": (I32, [P, I32, P, P, P]),
        "pic_state_bytes": (SZ, [P]),
        "pic_save_state": (I32, [P, P]),
        "pic_load_state": (I32, [P, P]),
        "pic_state_header_words": (I32, [P]),
        "pic_save_state_h": (I32, [P, P, P]),
        "pic_load_state_h": (I32, [P, P, P]),
        "pic_adjoint_set_particles": (I32, [P, P]),
        "pic_adjoint_get_particles": (I32, [P, P]),
        "pic_set_kernel_timing": (I32, [P, I32]),
        "pic_kernel_timing": (I32, [P, ctypes.POINTER(D)]),
        "pic_batch_workspace_bytes": (SZ, [cfgp, I32]),
        "pic_batch_create": (I32, [cfgp, I32, P, SZ, P, ctypes.POINTER(P)]),
        "pic_instance_count": (I32, [P]),
        "pic_graph_period": (I32, [P]),
        "pic_select_instance": (I32, [P, I32]),
        "step_batched": (I32, [P, I32]),
        "adjoint_seed_energy": (I32, [P, D, P]),
        "step_adjoint": (I32, [P, P, P]),
        "adjoint_initial": (I32, [P, P, P]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def make_config(nx, ny, lx, ly, dt, degree=3, scheme="bdf", bdf_order=2, dtype="f32",
                c=1.0, eps0=1.0, mu0=1.0, q=-1.0, m=1.0, max_particles=1, flags=0,
                sort_interval=0, tile_cells=0, chunk=0, slack=0):
    s = ConfigStruct()
    s.abi_version = PIC_ABI_VERSION
    s.nx, s.ny, s.spline_degree = nx, ny, degree
    s.lx, s.ly = lx, ly
    s.scheme, s.bdf_order = SCHEMES[scheme], bdf_order
    s.particle_dtype = DTYPES[dtype]
    s.sort_interval = sort_interval
    s.dt, s.c, s.eps0, s.mu0, s.q, s.m = dt, c, eps0, mu0, q, m
    s.max_particles = max_particles
    s.flags = flags
    s.tile_cells, s.chunk, s.slack = tile_cells, chunk, slack
    return s


def workspace_bytes(cfg):
    n = load().pic_workspace_bytes(ctypes.byref(cfg))
    if n == 0:
        raise PicError(1, load().pic_last_error(None).decode())
    return n


def history_fields(cfg):
    return load().pic_history_fields(ctypes.byref(cfg))


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr())


class Context:
    """Owns the torch workspace tensor and the libpic context.

    `cfg` is one ConfigStruct (plain) or a list of them (an ensemble)."""

    def __init__(self, cfg, device="cuda", stream=None):
        lib = load()
        cfgs = list(cfg) if isinstance(cfg, (list, tuple)) else [cfg]
        arr = (ConfigStruct * len(cfgs))(*cfgs)
        self.cfgs = cfgs
        self.cfg = cfgs[0]
        self.device = torch.device(device)
        if len(cfgs) == 1:
            nbytes = workspace_bytes(cfgs[0])
        else:
            nbytes = lib.pic_batch_workspace_bytes(arr, len(cfgs))
            if nbytes == 0:
                raise PicError(1, lib.pic_last_error(None).decode())
        self.workspace = torch.empty(nbytes + 256, dtype=torch.uint8, device=self.device)
        base = self.workspace.data_ptr()
        off = (-base) % 256
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        h = ctypes.c_void_p()
        if len(cfgs) == 1:
            st = lib.pic_create(ctypes.byref(cfgs[0]), ctypes.c_void_p(base + off), nbytes,
                                ctypes.c_void_p(self.stream.cuda_stream), ctypes.byref(h))
        else:
            st = lib.pic_batch_create(arr, len(cfgs), ctypes.c_void_p(base + off), nbytes,
                                      ctypes.c_void_p(self.stream.cuda_stream), ctypes.byref(h))
        if st != 0:
            raise PicError(st, lib.pic_last_error(None).decode())
        self.handle = h
        self.ns = [0] * len(cfgs)
        self.sel = 0

    @property
    def n(self):
        return self.ns[self.sel]

    @n.setter
    def n(self, v):
        self.ns[self.sel] = v

    def check(self, st):
        if st != 0:
            raise PicError(st, load().pic_last_error(self.handle).decode())

    def close(self):
        if getattr(self, "handle", None):
            load().pic_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def nx(self):
        return self.cfgs[self.sel].nx

    @property
    def ny(self):
        return self.cfgs[self.sel].ny


# ---------------------------------------------------------------------------
# entry points, named as in pic.h

def init_particles(ctx, x, y, P):
    """x, y: [n] float64; P: [3, n] float64 (CUDA tensors)."""
    n = x.numel()
    x = x.to(ctx.device, torch.float64).contiguous()
    y = y.to(ctx.device, torch.float64).contiguous()
    P = P.to(ctx.device, torch.float64).contiguous()
    assert y.numel() == n and P.numel() == 3 * n
    ctx._inputs = (x, y, P)  # kept alive until the stream has consumed them
    ctx.check(load().init_particles(ctx.handle, n, _ptr(x), _ptr(y), _ptr(P)))
    ctx.n = n


def deposit_current(ctx):
    ctx.check(load().deposit_current(ctx.handle))


def field_solve(ctx):
    ctx.check(load().field_solve(ctx.handle))


def gather_push(ctx):
    ctx.check(load().gather_push(ctx.handle))


def step(ctx, nsteps=1):
    ctx.check(load().step(ctx.handle, int(nsteps)))


def select_instance(ctx, index):
    ctx.check(load().pic_select_instance(ctx.handle, int(index)))
    ctx.sel = int(index)


def instance_count(ctx):
    return load().pic_instance_count(ctx.handle)


def graph_period(ctx):
    """Steps per replayed graph period (0: no graph replay); the first step()
    call of more steps than this captures the graph."""
    return load().pic_graph_period(ctx.handle)


def step_batched(ctx, nsteps=1):
    ctx.check(load().step_batched(ctx.handle, int(nsteps)))


def get_particles(ctx):
    out = torch.empty((11, ctx.n), dtype=torch.float64, device=ctx.device)
    ctx.check(load().pic_get_particles(ctx.handle, _ptr(out)))
    return out


def set_particles(ctx, parts):
    parts = parts.to(ctx.device, torch.float64).contiguous()
    assert parts.shape == (11, ctx.n)
    ctx._inputs = (parts,)
    ctx.check(load().pic_set_particles(ctx.handle, _ptr(parts)))


def j_planes(cfg):
    """Real J planes PIC_FIELD_J exports: 3, or 3 per DIRK stage when the
    stage currents are sub-stepped."""
    if cfg.flags & FLAG_DIRK_SUBSTEP:
        return 9 if cfg.scheme == SCHEMES["dirk3"] else 6
    return 3


def get_field(ctx, which):
    nf = j_planes(ctx.cfgs[ctx.sel]) if which == FIELD_J else 12
    out = torch.empty((nf, ctx.ny, ctx.nx), dtype=torch.float64, device=ctx.device)
    ctx.check(load().pic_get_field(ctx.handle, int(which), _ptr(out)))
    return out


def get_history(ctx):
    nf = history_fields(ctx.cfgs[ctx.sel])
    out = torch.empty((nf, ctx.ny, ctx.nx // 2 + 1), dtype=torch.complex128, device=ctx.device)
    ctx.check(load().pic_get_history(ctx.handle, _ptr(out)))
    return out


def set_history(ctx, hist):
    nf = history_fields(ctx.cfgs[ctx.sel])
    hist = hist.to(ctx.device, torch.complex128).contiguous()
    assert hist.shape == (nf, ctx.ny, ctx.nx // 2 + 1)
    ctx._inputs = (hist,)
    ctx.check(load().pic_set_history(ctx.handle, _ptr(hist)))


def diagnostics(ctx, allow_nonfinite=False):
    buf = (ctypes.c_double * 8)()
    st = load().pic_diagnostics(ctx.handle, buf)
    if st != 0 and not (allow_nonfinite and st == 6):
        ctx.check(st)
    return dict(zip(DIAG_NAMES, list(buf)))


class State:
    """A device buffer holding one saved state of a context (pic_save_state),
    with a host copy of its header (pic_save_state_h)."""

    def __init__(self, ctx):
        nbytes = load().pic_state_bytes(ctx.handle)
        self.buf = torch.empty(nbytes + 256, dtype=torch.uint8, device=ctx.device)
        self.ptr = ctypes.c_void_p(self.buf.data_ptr() + (-self.buf.data_ptr()) % 256)
        self.header = (ctypes.c_int64 * load().pic_state_header_words(ctx.handle))()
        self.ns = None


def save_state(ctx, state=None):
    """Save the context's state (phase READY or SOLVED) into `state` (a new State if None)."""
    state = state or State(ctx)
    ctx.check(load().pic_save_state_h(ctx.handle, state.ptr, ctypes.cast(state.header, ctypes.c_void_p)))
    state.ns = list(ctx.ns)
    return state


def load_state(ctx, state, trust_header=False):
    """Restore `state`.  trust_header: take the header saved with it on the
    host (pic_load_state_h: no read of the buffer, no synchronisation); only
    for a State whose buffer nothing else wrote since save_state."""
    if trust_header:
        if len(state.header) != load().pic_state_header_words(ctx.handle):
            raise ValueError("the state's header does not fit this context")
        ctx.check(load().pic_load_state_h(ctx.handle, state.ptr, ctypes.cast(state.header, ctypes.c_void_p)))
    else:
        ctx.check(load().pic_load_state(ctx.handle, state.ptr))
    ctx.ns = list(state.ns)


def set_dirk_tableau(ctx, A, b, c):
    """Replace the DIRK tableau (A: s x s lower triangular, b, c: length s;
    host values)."""
    import numpy as np
    A = np.ascontiguousarray(A, np.float64)
    b = np.ascontiguousarray(b, np.float64)
    c = np.ascontiguousarray(c, np.float64)
    ctx.check(load().pic_set_dirk_tableau(ctx.handle, b.shape[0], ctypes.c_void_p(A.ctypes.data),
                                          ctypes.c_void_p(b.ctypes.data), ctypes.c_void_p(c.ctypes.data)))


def diagnostics_all(ctx):
    """pic_diagnostics of every instance into a device tensor [ninst, 8] (the
    DIAG_NAMES order), enqueued on the context's stream without allocation in
    the library and without synchronisation."""
    out = torch.empty((instance_count(ctx), 8), dtype=torch.float64, device=ctx.device)
    ctx.check(load().pic_diagnostics_all(ctx.handle, _ptr(out)))
    return out


def set_kernel_timing(ctx, enable=True):
    ctx.check(load().pic_set_kernel_timing(ctx.handle, 1 if enable else 0))


def kernel_timing(ctx):
    """{class: (total ms, launches)} since the last call (synchronises)."""
    buf = (ctypes.c_double * (2 * len(KCLASSES)))()
    ctx.check(load().pic_kernel_timing(ctx.handle, buf))
    return {k: (buf[2 * i], int(buf[2 * i + 1])) for i, k in enumerate(KCLASSES)}


def adjoint_seed_energy(ctx, scale=1.0):
    """d(scale * field energy)/d(history) as a complex [nf, ny, nx/2+1] tensor."""
    nf = history_fields(ctx.cfgs[ctx.sel])
    out = torch.empty((nf, ctx.ny, ctx.nx // 2 + 1), dtype=torch.complex128, device=ctx.device)
    ctx.check(load().adjoint_seed_energy(ctx.handle, float(scale), _ptr(out)))
    return out


def step_adjoint(ctx, lam, lam_hist):
    """lambda^{n+1} -> lambda^n in place; the context must hold S^n (phase READY).
    lam None: the particle adjoint the context holds (adjoint_set_particles)."""
    if lam is not None:
        assert lam.dtype == torch.float64 and lam.is_contiguous() and lam.shape == (11, ctx.n)
    assert lam_hist.dtype == torch.complex128 and lam_hist.is_contiguous()
    assert lam_hist.shape == (history_fields(ctx.cfgs[ctx.sel]), ctx.ny, ctx.nx // 2 + 1)
    ctx.check(load().step_adjoint(ctx.handle, None if lam is None else _ptr(lam), _ptr(lam_hist)))


def adjoint_set_particles(ctx, lam=None):
    """Hold lam [11, n] (original order; None: zero) as the context's particle adjoint."""
    if lam is not None:
        assert lam.dtype == torch.float64 and lam.is_contiguous() and lam.shape == (11, ctx.n)
        ctx._inputs = (lam,)
    ctx.check(load().pic_adjoint_set_particles(ctx.handle, None if lam is None else _ptr(lam)))


def adjoint_get_particles(ctx):
    """The held particle adjoint as [11, n] float64 in original order."""
    out = torch.empty((11, ctx.n), dtype=torch.float64, device=ctx.device)
    ctx.check(load().pic_adjoint_get_particles(ctx.handle, _ptr(out)))
    return out


def adjoint_initial(ctx, P0, lam):
    """Fold the adjoint of v^0 = v^{-1} = V(P0) into lam[2:5] (in place)."""
    P0 = P0.to(ctx.device, torch.float64).contiguous()
    assert P0.numel() == 3 * ctx.n and lam.shape == (11, ctx.n) and lam.is_contiguous()
    ctx._inputs = (P0,)
    ctx.check(load().adjoint_initial(ctx.handle, _ptr(P0), _ptr(lam)))
