"""ctypes binding of libgpf.so (include/gpf.h).

Argument marshalling only: every step of a solve runs in the library's HIP
kernels.  torch tensors supply device memory and streams.  Importing this
module loads the in-tree library and raises if it has not been built.
"""
from __future__ import annotations

import ctypes as C
import math
import os
import re

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libgpf.so")
HEADER = os.path.join(os.path.dirname(HERE), "include", "gpf.h")

GPF_OK = 0
GPF_E_INVALID = -1
GPF_E_OUT_OF_GRID = -2
GPF_E_SINGULAR = -3
GPF_E_NOMEM = -4
GPF_E_DEVICE = -5
GPF_E_UNSUPPORTED = -6
GPF_E_BUSY = -7
STATUS_NAMES = {0: "GPF_OK", -1: "GPF_E_INVALID", -2: "GPF_E_OUT_OF_GRID", -3: "GPF_E_SINGULAR",
                -4: "GPF_E_NOMEM", -5: "GPF_E_DEVICE", -6: "GPF_E_UNSUPPORTED", -7: "GPF_E_BUSY"}

GPF_DEV_OUT_OF_GRID = 1
GPF_DEV_SINGULAR = 2

GPF_FP32 = 0
GPF_FP64 = 1
GPF_CONV1_FP64 = 2
GPF_POLICY_AUTO = 4
GPF_PSI_TOTAL = 8
GPF_PLAN_MULTISTREAM = 16

TK_NAMES = ["scatter", "rows_fwd", "cols", "rows_inv", "rows_fwd64", "cols64", "rows_inv64",
            "surface", "velocity"]

GPF_NOBODY, GPF_CIRCULATION, GPF_KUTTA_STEADY, GPF_KUTTA_SHED = 0, 1, 2, 3
MODES = {"none": GPF_NOBODY, "circulation": GPF_CIRCULATION, "kutta": GPF_KUTTA_STEADY,
         "shed": GPF_KUTTA_SHED}
GPF_MAX_EDGES = 8
N_SCALARS = 4 + GPF_MAX_EDGES + 2 * 8


class GpfError(RuntimeError):
    def __init__(self, status: int, where: str, msg: str):
        super().__init__(f"{where}: {STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


class gpf_grid(C.Structure):
    _fields_ = [("n", C.c_int), ("dx", C.c_double), ("x0", C.c_double), ("y0", C.c_double)]


class gpf_schedule(C.Structure):
    _fields_ = [("rows", C.c_int), ("order", C.c_int), ("cols", C.c_int)]


GPF_PARTS = 4
GPF_MAX_PARTS = 8


class gpf_part(C.Structure):
    _fields_ = [("mode", C.c_int), ("gamma_b", C.c_double), ("gamma_w", C.c_double),
                ("ub", C.c_double), ("vb", C.c_double), ("omega", C.c_double)]


class gpf_inputs(C.Structure):
    _fields_ = [("nv", C.c_int), ("d_xv", C.c_void_p), ("d_yv", C.c_void_p), ("d_gv", C.c_void_p),
                ("u_inf", C.c_double), ("v_inf", C.c_double),
                ("ub", C.c_double), ("vb", C.c_double), ("omega", C.c_double),
                ("mode", C.c_int), ("gamma_b", C.c_double), ("m", C.c_int),
                ("h_xnew", C.c_double * GPF_MAX_EDGES), ("h_ynew", C.c_double * GPF_MAX_EDGES),
                ("gamma_w", C.c_double),
                ("fmin", C.c_double * GPF_MAX_EDGES), ("fmax", C.c_double * GPF_MAX_EDGES),
                ("nparts", C.c_int), ("parts", gpf_part * GPF_MAX_PARTS)]


class gpf_outputs(C.Structure):
    _fields_ = [("d_psi", C.c_void_p), ("d_u", C.c_void_p), ("d_v", C.c_void_p),
                ("d_f", C.c_void_p), ("d_ftilde", C.c_void_p), ("d_scalars", C.c_void_p),
                ("d_status", C.c_void_p), ("d_impulse", C.c_void_p)]


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with __graft_entry__.build()")
    # torch's HIP runtime must be the one the library binds to: both carry
    # the soname libamdhip64.so.7, but torch loads its copy by file name, so
    # loading the library first would put two HIP runtimes in the process.
    import torch  # noqa: F401
    lib = C.CDLL(LIB_PATH)
    P = C.c_void_p
    PP = C.POINTER(C.c_void_p)
    D = C.c_double
    I = C.c_int
    DP = C.POINTER(C.c_double)
    sig = {
        "gpf_ctx_create": (I, [I, PP]),
        "gpf_ctx_destroy": (None, [P]),
        "gpf_plan_create": (I, [P, C.POINTER(gpf_grid), C.c_uint, PP]),
        "gpf_plan_destroy": (None, [P]),
        "gpf_body_create": (I, [P, I, DP, DP, DP, I, C.POINTER(C.c_int), PP]),
        "gpf_body_destroy": (None, [P]),
        "gpf_body_info": (I, [P, DP, DP, C.POINTER(C.c_int)]),
        "gpf_body_f0": (I, [P, DP]),
        "gpf_body_set_normals": (I, [P, DP, DP, I]),
        "gpf_pressure": (I, [P, P, C.POINTER(gpf_inputs), P, P, P, D, D, P, P, P, P, P]),
        "gpf_body_geometry": (I, [P, DP, DP, DP]),
        "gpf_body_added_mass": (I, [P, D, DP]),
        "gpf_body_set_parts": (I, [P, I, C.POINTER(C.c_int)]),
        "gpf_body_schur_by_convolution": (I, [P, I, I, DP, DP, DP]),
        "gpf_solve": (I, [P, P, C.POINTER(gpf_inputs), C.POINTER(gpf_outputs), P]),
        "gpf_regularize_vortices": (I, [P, I, P, P, P, P, I, P, P]),
        "gpf_convolve": (I, [P, P, P, D, P]),
        "gpf_convolve_noalloc": (I, [P, P, P, D, P]),
        "gpf_interpolate_surface": (I, [P, P, P, P]),
        "gpf_vortex_velocity": (I, [P, P, I, P, P, D, D, P, P, P, P]),
        "gpf_lgf_table": (I, [I, DP]),
        "gpf_invert_fp64": (I, [P, I, P, P, P, DP]),
        "gpf_schedule_set": (I, [P, I, I, I, C.POINTER(gpf_schedule)]),
        "gpf_schedule_get": (I, [P, I, I, I, C.POINTER(gpf_schedule)]),
        "gpf_autotune": (I, [P, I, I, C.c_char_p, C.POINTER(gpf_schedule), DP]),
        "gpf_autotune_batched": (I, [P, I, C.POINTER(C.c_void_p), C.POINTER(C.c_void_p),
                                     C.POINTER(gpf_inputs), C.POINTER(gpf_outputs), P]),
        "gpf_timing_enable": (I, [P, I]),
        "gpf_timing_read": (I, [P, I, C.POINTER(C.c_longlong), DP]),
        "gpf_batch_create": (I, [P, I, PP]),
        "gpf_batch_destroy": (None, [P]),
        "gpf_batch_set_lanes": (I, [P, I]),
        "gpf_batch_get_lanes": (I, [P]),
        "gpf_batch_set_merge": (I, [P, I]),
        "gpf_solve_batched": (I, [P, I, C.POINTER(C.c_void_p), C.POINTER(C.c_void_p),
                                  C.POINTER(gpf_inputs), C.POINTER(gpf_outputs), P]),
        "gpf_rk2_create": (I, [P, P, C.POINTER(gpf_inputs), P, P, D, I, PP]),
        "gpf_rk2_run": (I, [P, I, P]),
        "gpf_rk2_fields": (I, [P, PP, PP, PP, PP, PP, PP]),
        "gpf_rk2_destroy": (None, [P]),
        "gpf_shed_create": (I, [P, P, C.POINTER(gpf_inputs), C.POINTER(gpf_outputs), P, P, P, I,
                                D, DP, PP]),
        "gpf_shed_run": (I, [P, I, P]),
        "gpf_shed_count": (I, [P]),
        "gpf_shed_destroy": (None, [P]),
        "gpf_server_create": (I, [P, C.c_size_t, I, C.c_uint, PP]),
        "gpf_server_plan": (I, [P, C.POINTER(gpf_grid), PP]),
        "gpf_server_submit": (I, [P, C.POINTER(gpf_grid), P, C.POINTER(gpf_inputs),
                                  C.POINTER(gpf_outputs), C.POINTER(C.c_ulonglong)]),
        "gpf_server_poll": (I, [P, C.c_ulonglong, C.POINTER(C.c_int), DP]),
        "gpf_server_wait": (I, [P, C.c_ulonglong, DP]),
        "gpf_server_destroy": (None, [P]),
        "gpf_server_stats": (I, [P, C.POINTER(C.c_ulonglong), C.POINTER(C.c_int)]),
        "gpf_sync": (I, [P, P]),
        "gpf_last_error": (C.c_char_p, []),
        "gpf_version": (C.c_char_p, []),
    }
    for name, (res, args) in sig.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    return lib


lib = _load()


def declared_symbols() -> list[str]:
    """Names of the functions declared in include/gpf.h."""
    with open(HEADER) as fh:
        text = fh.read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(gpf_[a-z0-9_]+)\s*\(", text)))


def check(st: int, where: str) -> None:
    if st != GPF_OK:
        raise GpfError(st, where, lib.gpf_last_error().decode())


def _dp(arr):
    import numpy as np
    a = np.ascontiguousarray(arr, dtype=np.float64)
    return a, a.ctypes.data_as(C.POINTER(C.c_double))


def lgf_table(nmax: int):
    """Host lattice Green's function table from the library (no GPU needed)."""
    import numpy as np
    t = np.zeros((nmax + 1) * (nmax + 1))
    check(lib.gpf_lgf_table(nmax, t.ctypes.data_as(C.POINTER(C.c_double))), "gpf_lgf_table")
    return t.reshape(nmax + 1, nmax + 1)


# ---------------------------------------------------------------------------
# object wrappers (torch supplies device memory and streams)
# ---------------------------------------------------------------------------

def _stream_ptr(stream=None):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return C.c_void_p(s.cuda_stream)


def _ptr(t):
    return None if t is None else C.c_void_p(t.data_ptr())


class Context:
    def __init__(self, device: int = 0):
        h = C.c_void_p()
        check(lib.gpf_ctx_create(device, C.byref(h)), "gpf_ctx_create")
        self.h = h
        self.device = device

    def close(self):
        if self.h:
            lib.gpf_ctx_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Plan:
    def __init__(self, ctx: Context, n: int, dx: float, x0: float | None = None,
                 y0: float | None = None, flags: int = GPF_FP32, _handle=None):
        if x0 is None:
            x0 = -(n - 1) * dx / 2.0
        if y0 is None:
            y0 = -(n - 1) * dx / 2.0
        self.ctx = ctx
        self.n, self.dx, self.x0, self.y0, self.flags = n, dx, x0, y0, flags
        self.fp64 = bool(flags & GPF_FP64)
        self.grid = gpf_grid(n, dx, x0, y0)
        self.owned = _handle is None
        if _handle is not None:     # a plan owned by a server
            self.h = _handle
            return
        h = C.c_void_p()
        check(lib.gpf_plan_create(ctx.h, C.byref(self.grid), flags, C.byref(h)), "gpf_plan_create")
        self.h = h

    @property
    def field_dtype(self):
        import torch
        return torch.float64 if self.fp64 else torch.float32

    def close(self):
        if self.h and self.owned:
            lib.gpf_plan_destroy(self.h)
        self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Body:
    def __init__(self, plan: Plan, xs, ys, ds, edges=()):
        self.plan = plan
        ax, px = _dp(xs)
        ay, py = _dp(ys)
        ad, pd = _dp(ds)
        self.ns = len(ax)
        self.edges = tuple(int(e) for e in edges)
        ed = (C.c_int * max(1, len(self.edges)))(*self.edges)
        h = C.c_void_p()
        check(lib.gpf_body_create(plan.h, self.ns, px, py, pd, len(self.edges), ed, C.byref(h)),
              "gpf_body_create")
        self.h = h

    def info(self):
        g0, amp, c1 = C.c_double(), C.c_double(), C.c_int()
        check(lib.gpf_body_info(self.h, C.byref(g0), C.byref(amp), C.byref(c1)), "gpf_body_info")
        return {"gamma0": g0.value, "amp": amp.value, "conv1_fp64": bool(c1.value)}

    def f0(self):
        import numpy as np
        out = np.zeros(self.ns)
        check(lib.gpf_body_f0(self.h, out.ctypes.data_as(C.POINTER(C.c_double))), "gpf_body_f0")
        return out

    def set_normals(self, nx, ny, closed: bool = True):
        """Unit normals; closed=False for a zero-thickness body (a plate)."""
        ax, px = _dp(nx)
        ay, py = _dp(ny)
        assert len(ax) == len(ay) == self.ns
        check(lib.gpf_body_set_normals(self.h, px, py, int(bool(closed))), "gpf_body_set_normals")

    def set_parts(self, part):
        """Split the points into parts: part[p] = part of point p."""
        import numpy as np
        a = np.ascontiguousarray(np.asarray(part, dtype=np.int32))
        assert len(a) == self.ns
        self.nparts = int(a.max()) + 1
        check(lib.gpf_body_set_parts(self.h, self.nparts, a.ctypes.data_as(C.POINTER(C.c_int))),
              "gpf_body_set_parts")

    def geometry(self):
        """(area, x_c, y_c)."""
        v = [C.c_double() for _ in range(3)]
        check(lib.gpf_body_geometry(self.h, *[C.byref(a) for a in v]), "gpf_body_geometry")
        return tuple(a.value for a in v)

    def added_mass(self, rho: float = 1.0):
        """3x3 added-mass tensor (rows: x, y, rotation; columns: F_x, F_y, M)."""
        import numpy as np
        out = np.zeros(9)
        check(lib.gpf_body_added_mass(self.h, float(rho), out.ctypes.data_as(C.POINTER(C.c_double))),
              "gpf_body_added_mass")
        return out.reshape(3, 3)

    def schur_by_convolution(self, fp64: bool = False, batch: int = 32):
        """S built column by column from batched unit sheets, against the
        exact S: (relative Frobenius error of S, relative error of the unit
        uniform-flow sheet, build time in ms)."""
        v = [C.c_double() for _ in range(3)]
        check(lib.gpf_body_schur_by_convolution(self.h, int(bool(fp64)), int(batch),
                                                *[C.byref(a) for a in v]),
              "gpf_body_schur_by_convolution")
        return tuple(a.value for a in v)

    def close(self):
        if self.h:
            lib.gpf_body_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def make_inputs(X, Y, G, u_inf=0.0, v_inf=0.0, ub=0.0, vb=0.0, omega=0.0, mode="none",
                gamma_b=0.0, znew=(), gamma_w=None, fbounds=()) -> gpf_inputs:
    """Fill gpf_inputs; X, Y, G are float64 device tensors.  fbounds:
    ((fmin, fmax), ...) per edge for the shedding mode; () is Kutta."""
    inp = gpf_inputs()
    inp.nv = int(X.numel()) if X is not None else 0
    inp.d_xv = X.data_ptr() if inp.nv else None
    inp.d_yv = Y.data_ptr() if inp.nv else None
    inp.d_gv = G.data_ptr() if inp.nv else None
    inp.u_inf, inp.v_inf, inp.ub, inp.vb, inp.omega = u_inf, v_inf, ub, vb, omega
    inp.mode = MODES[mode] if isinstance(mode, str) else int(mode)
    inp.gamma_b = gamma_b
    inp.m = len(znew)
    for j, z in enumerate(znew):
        inp.h_xnew[j] = z[0]
        inp.h_ynew[j] = z[1]
    inp.gamma_w = math.nan if gamma_w is None else gamma_w
    for j, (lo, hi) in enumerate(fbounds):
        inp.fmin[j] = lo
        inp.fmax[j] = hi
    return inp


def make_parts_inputs(X, Y, G, parts, znew=(), fbounds=(), u_inf=0.0, v_inf=0.0) -> gpf_inputs:
    """gpf_inputs for mode GPF_PARTS.  parts: one dict per part with keys
    mode ("circulation" | "kutta" | "shed"), and optionally gamma_b,
    gamma_w, ub, vb, omega; znew / fbounds: one entry per edge of the
    shedding parts, in the body's edge order."""
    inp = make_inputs(X, Y, G, u_inf, v_inf, mode=GPF_PARTS, znew=znew, fbounds=fbounds)
    inp.nparts = len(parts)
    for j, q in enumerate(parts):
        inp.parts[j].mode = MODES[q["mode"]]
        inp.parts[j].gamma_b = q.get("gamma_b", 0.0)
        inp.parts[j].gamma_w = q.get("gamma_w", 0.0)
        inp.parts[j].ub = q.get("ub", 0.0)
        inp.parts[j].vb = q.get("vb", 0.0)
        inp.parts[j].omega = q.get("omega", 0.0)
    return inp


def gpf_pressure(plan: Plan, body: Body, inp: gpf_inputs, psi, f, dphi, dp, p=None, pside=None,
                 dphi_prev=None, dt: float = 0.0, rho: float = 1.0, stream=None):
    """Pressure of a solved problem into the given device tensors."""
    check(lib.gpf_pressure(plan.h, body.h, C.byref(inp), _ptr(psi), _ptr(f),
                           None if dphi_prev is None else _ptr(dphi_prev), float(dt), float(rho),
                           _ptr(dphi), _ptr(dp), None if p is None else _ptr(p),
                           None if pside is None else _ptr(pside), _stream_ptr(stream)),
          "gpf_pressure")


def make_outputs(psi, u=None, v=None, f=None, ftilde=None, scalars=None, status=None,
                 impulse=None) -> gpf_outputs:
    out = gpf_outputs()
    out.d_psi = psi.data_ptr()
    out.d_u = None if u is None else u.data_ptr()
    out.d_v = None if v is None else v.data_ptr()
    out.d_f = None if f is None else f.data_ptr()
    out.d_ftilde = None if ftilde is None else ftilde.data_ptr()
    out.d_scalars = None if scalars is None else scalars.data_ptr()
    out.d_status = status.data_ptr()
    out.d_impulse = None if impulse is None else impulse.data_ptr()
    return out


class Outputs:
    """Device tensors for one solve's outputs (field of the plan's type, FP64
    velocities, surface strengths and scalars) and their gpf_outputs."""

    def __init__(self, n: int, nv: int, ns: int = 0, fp64: bool = False, device=None):
        import torch
        dev = device or torch.device("cuda", 0)
        self.psi = torch.empty((n, n), dtype=torch.float64 if fp64 else torch.float32, device=dev)
        self.u = torch.empty(max(nv, 1), dtype=torch.float64, device=dev)
        self.v = torch.empty_like(self.u)
        self.f = torch.empty(max(ns, 1), dtype=torch.float64, device=dev) if ns else None
        self.ft = torch.empty_like(self.f) if ns else None
        self.scalars = torch.zeros(N_SCALARS, dtype=torch.float64, device=dev)
        self.status = torch.zeros(1, dtype=torch.int32, device=dev)
        # the clears are done before any stream (the server's are non-blocking) writes
        torch.cuda.current_stream(dev).synchronize()
        self.struct = make_outputs(self.psi, self.u if nv else None, self.v if nv else None,
                                   self.f, self.ft, self.scalars, self.status)


def gpf_solve(plan: Plan, body: Body | None, inp: gpf_inputs, out: gpf_outputs, stream=None):
    check(lib.gpf_solve(plan.h, None if body is None else body.h, C.byref(inp), C.byref(out),
                        _stream_ptr(stream)), "gpf_solve")


def schedule_set(ctx: Context, n: int, fp64: bool, nb: int, sched=None):
    """sched: {"rows", "order", "cols"} or None (back to the rules)."""
    ptr = None
    if sched is not None:
        ptr = C.byref(gpf_schedule(int(sched["rows"]), int(sched["order"]), int(sched["cols"])))
    check(lib.gpf_schedule_set(ctx.h, int(n), int(bool(fp64)), int(nb), ptr), "gpf_schedule_set")


def schedule_get(ctx: Context, n: int, fp64: bool, nb: int) -> dict:
    g = gpf_schedule()
    check(lib.gpf_schedule_get(ctx.h, int(n), int(bool(fp64)), int(nb), C.byref(g)),
          "gpf_schedule_get")
    return {"rows": g.rows, "order": g.order, "cols": g.cols}


def autotune(plan: Plan, fp64: bool, nb: int, cache_path=None):
    """Time the convolution schedules for nb problems of the plan's grid;
    returns (chosen schedule, microseconds per batched convolution)."""
    g, us = gpf_schedule(), C.c_double()
    path = None if cache_path is None else os.fsencode(cache_path)
    check(lib.gpf_autotune(plan.h, int(bool(fp64)), int(nb), path, C.byref(g), C.byref(us)),
          "gpf_autotune")
    return {"rows": g.rows, "order": g.order, "cols": g.cols}, us.value


def timing_enable(plan: Plan, enable: bool = True):
    check(lib.gpf_timing_enable(plan.h, int(bool(enable))), "gpf_timing_enable")


def timing_read(plan: Plan) -> dict:
    """{kernel class: (launch count, total ms)}; waits for the events."""
    out = {}
    for k, name in enumerate(TK_NAMES):
        cnt, ms = C.c_longlong(), C.c_double()
        check(lib.gpf_timing_read(plan.h, k, C.byref(cnt), C.byref(ms)), "gpf_timing_read")
        out[name] = (cnt.value, ms.value)
    return out


def gpf_sync(status, stream=None):
    check(lib.gpf_sync(_stream_ptr(stream), C.c_void_p(status.data_ptr())), "gpf_sync")


def gpf_regularize_vortices(plan: Plan, X, Y, G, w, accumulate=False, status=None, stream=None):
    nv = int(X.numel())
    check(lib.gpf_regularize_vortices(plan.h, nv, _ptr(X) if nv else None, _ptr(Y) if nv else None,
                                      _ptr(G) if nv else None, _ptr(w), int(bool(accumulate)),
                                      _ptr(status), _stream_ptr(stream)), "gpf_regularize_vortices")


def gpf_convolve(plan: Plan, w, s, gamma_src: float, stream=None):
    check(lib.gpf_convolve(plan.h, _ptr(w), _ptr(s), float(gamma_src), _stream_ptr(stream)),
          "gpf_convolve")


def gpf_convolve_noalloc(plan: Plan, w, s, gamma_src: float, stream=None):
    check(lib.gpf_convolve_noalloc(plan.h, _ptr(w), _ptr(s), float(gamma_src),
                                   _stream_ptr(stream)), "gpf_convolve_noalloc")


def gpf_invert_fp64(ctx: Context, a, ainv, stream=None) -> float:
    """ainv = a^-1 for a square FP64 device tensor (row-major, contiguous);
    returns min |pivot| / max |a_ij|."""
    n = int(a.shape[0])
    mp = C.c_double(0.0)
    check(lib.gpf_invert_fp64(ctx.h, n, _ptr(a), _ptr(ainv), _stream_ptr(stream), C.byref(mp)),
          "gpf_invert_fp64")
    return mp.value


def gpf_interpolate_surface(body: Body, s, r, stream=None):
    check(lib.gpf_interpolate_surface(body.h, _ptr(s), _ptr(r), _stream_ptr(stream)),
          "gpf_interpolate_surface")


def gpf_vortex_velocity(plan: Plan, s, X, Y, u_inf, v_inf, u, v, status=None, stream=None):
    nv = int(X.numel())
    check(lib.gpf_vortex_velocity(plan.h, _ptr(s), nv, _ptr(X), _ptr(Y), float(u_inf),
                                  float(v_inf), _ptr(u), _ptr(v), _ptr(status),
                                  _stream_ptr(stream)), "gpf_vortex_velocity")


class Batch:
    """Workspaces for up to max_problems problems solved in shared launches."""

    def __init__(self, ctx: Context, max_problems: int, lanes: int = 1, merge: int = 1):
        h = C.c_void_p()
        check(lib.gpf_batch_create(ctx.h, max_problems, C.byref(h)), "gpf_batch_create")
        self.h = h
        self.ctx = ctx
        self.max_problems = max_problems
        if lanes != 1:
            check(lib.gpf_batch_set_lanes(h, int(lanes)), "gpf_batch_set_lanes")
        self.lanes = lanes
        self.merge = 1
        if int(merge) != 1:
            self.set_merge(merge)

    def set_merge(self, merge: int):
        """0: group by group; 1: merged, FP64-first-convolution problems on a
        side stream; 2: merged on the caller's stream alone (gpf_batch_set_merge)."""
        check(lib.gpf_batch_set_merge(self.h, int(merge)), "gpf_batch_set_merge")
        self.merge = int(merge)

    def solve(self, plans, bodies, inputs, outputs, stream=None):
        k = len(plans)
        pa = (C.c_void_p * k)(*[p.h.value for p in plans])
        ba = (C.c_void_p * k)(*[(b.h.value if b is not None else None) for b in bodies])
        ia = (gpf_inputs * k)(*inputs)
        oa = (gpf_outputs * k)(*outputs)
        check(lib.gpf_solve_batched(self.h, k, pa, ba, ia, oa, _stream_ptr(stream)),
              "gpf_solve_batched")

    def autotune(self, plans, bodies, inputs, outputs, stream=None):
        """Choose the lane count and the convolution schedules of this
        workload by timing the batched solve under each
        (gpf_autotune_batched); the outputs then hold the result of the last
        solve, and self.lanes the chosen lane count."""
        k = len(plans)
        pa = (C.c_void_p * k)(*[p.h.value for p in plans])
        ba = (C.c_void_p * k)(*[(b.h.value if b is not None else None) for b in bodies])
        ia = (gpf_inputs * k)(*inputs)
        oa = (gpf_outputs * k)(*outputs)
        check(lib.gpf_autotune_batched(self.h, k, pa, ba, ia, oa, _stream_ptr(stream)),
              "gpf_autotune_batched")
        self.lanes = int(lib.gpf_batch_get_lanes(self.h))

    def close(self):
        if self.h:
            lib.gpf_batch_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Server:
    """Request server (gpf_server_*): resident plans per grid, batches of up
    to max_slots queued requests solved by a worker thread."""

    def __init__(self, ctx: Context, hbm_budget_bytes: int, max_slots: int, flags: int = GPF_POLICY_AUTO):
        h = C.c_void_p()
        check(lib.gpf_server_create(ctx.h, int(hbm_budget_bytes), int(max_slots), flags, C.byref(h)),
              "gpf_server_create")
        self.h, self.ctx, self.flags = h, ctx, flags
        self._plans = {}

    def plan(self, n: int, dx: float, x0: float | None = None, y0: float | None = None) -> Plan:
        x0 = -(n - 1) * dx / 2.0 if x0 is None else x0
        y0 = -(n - 1) * dx / 2.0 if y0 is None else y0
        key = (n, dx, x0, y0)
        if key not in self._plans:
            g = gpf_grid(n, dx, x0, y0)
            h = C.c_void_p()
            check(lib.gpf_server_plan(self.h, C.byref(g), C.byref(h)), "gpf_server_plan")
            self._plans[key] = Plan(self.ctx, n, dx, x0, y0, self.flags, _handle=h)
        return self._plans[key]

    def submit(self, plan: Plan, body, inp: gpf_inputs, out: gpf_outputs) -> int:
        rid = C.c_ulonglong()
        check(lib.gpf_server_submit(self.h, C.byref(plan.grid), None if body is None else body.h,
                                    C.byref(inp), C.byref(out), C.byref(rid)), "gpf_server_submit")
        return rid.value

    def poll(self, rid: int):
        """(done, latency_s or None)"""
        done, lat = C.c_int(), C.c_double()
        check(lib.gpf_server_poll(self.h, rid, C.byref(done), C.byref(lat)), "gpf_server_poll")
        return bool(done.value), (lat.value if done.value else None)

    def wait(self, rid: int) -> float:
        lat = C.c_double()
        check(lib.gpf_server_wait(self.h, rid, C.byref(lat)), "gpf_server_wait")
        return lat.value

    def stats(self):
        """(batches dispatched, most batches in flight at once)"""
        b, m = C.c_ulonglong(), C.c_int()
        check(lib.gpf_server_stats(self.h, C.byref(b), C.byref(m)), "gpf_server_stats")
        return b.value, m.value

    def close(self):
        if self.h:
            for p in self._plans.values():
                p.h = None
            lib.gpf_server_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Rk2:
    """Explicit-midpoint vortex advection; X, Y (float64 device tensors) are
    updated in place by run()."""

    def __init__(self, plan: Plan, body, inp: gpf_inputs, X, Y, dt: float, use_graph=True):
        h = C.c_void_p()
        check(lib.gpf_rk2_create(plan.h, None if body is None else body.h, C.byref(inp),
                                 _ptr(X), _ptr(Y), float(dt), int(bool(use_graph)), C.byref(h)),
              "gpf_rk2_create")
        self.h = h
        self.plan, self.body, self.inp, self.X, self.Y = plan, body, inp, X, Y

    def run(self, nsteps: int, stream=None):
        check(lib.gpf_rk2_run(self.h, int(nsteps), _stream_ptr(stream)), "gpf_rk2_run")

    def status_ptr(self) -> int:
        ptrs = [C.c_void_p() for _ in range(6)]
        check(lib.gpf_rk2_fields(self.h, *[C.byref(p) for p in ptrs]), "gpf_rk2_fields")
        return ptrs[5].value

    def sync(self, stream=None):
        check(lib.gpf_sync(_stream_ptr(stream), C.c_void_p(self.status_ptr())), "gpf_sync")

    def close(self):
        if self.h:
            lib.gpf_rk2_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Shed:
    """Vortex shedding with forward Euler steps.  X, Y, G are float64 device
    tensors of `capacity` entries whose first inp.nv hold the initial
    vortices; run() appends one vortex per edge each step and moves them all
    in place.  out: gpf_outputs with u, v of `capacity` entries, scalars and
    status.  first: ((dx, dy), ...) offset of each shedding edge's first
    release.  inp may be a GPF_PARTS input (several bodies): then every edge
    of a shedding part sheds, in body edge order."""

    def __init__(self, plan: Plan, body: Body, inp: gpf_inputs, out: gpf_outputs, X, Y, G,
                 dt: float, first):
        assert X.numel() == Y.numel() == G.numel()
        h = C.c_void_p()
        arr = (C.c_double * (2 * len(first)))(*[float(c) for z in first for c in z])
        check(lib.gpf_shed_create(plan.h, body.h, C.byref(inp), C.byref(out), _ptr(X), _ptr(Y),
                                  _ptr(G), int(X.numel()), float(dt), arr, C.byref(h)),
              "gpf_shed_create")
        self.h = h
        self.plan, self.body, self.inp, self.out, self.X, self.Y, self.G = \
            plan, body, inp, out, X, Y, G

    def run(self, nsteps: int, stream=None):
        check(lib.gpf_shed_run(self.h, int(nsteps), _stream_ptr(stream)), "gpf_shed_run")

    @property
    def nv(self) -> int:
        return lib.gpf_shed_count(self.h)

    def sync(self, stream=None):
        check(lib.gpf_sync(_stream_ptr(stream), C.c_void_p(self.out.d_status)), "gpf_sync")

    def close(self):
        if self.h:
            lib.gpf_shed_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Solver:
    """One plan (and optional body) with preallocated torch outputs.

    solve() runs gpf_solve and returns the output tensors (device).
    """

    def __init__(self, ctx: Context, n: int, dx: float, surface=None, flags: int = GPF_FP32,
                 edges=None):
        import torch
        self.plan = Plan(ctx, n, dx, flags=flags)
        self.body = None
        dev = torch.device("cuda", ctx.device)
        self.dev = dev
        if surface is not None:
            self.body = Body(self.plan, surface.xs, surface.ys, surface.ds,
                             surface.edges if edges is None else edges)
        ns = self.body.ns if self.body else 1
        self.psi = torch.empty((n, n), dtype=self.plan.field_dtype, device=dev)
        self.f = torch.zeros(ns, dtype=torch.float64, device=dev)
        self.ftilde = torch.zeros(ns, dtype=torch.float64, device=dev)
        self.scalars = torch.zeros(N_SCALARS, dtype=torch.float64, device=dev)
        self.status = torch.zeros(1, dtype=torch.int32, device=dev)
        self.u = self.v = None

    def upload(self, case):
        import torch
        t = lambda a: torch.as_tensor(a, dtype=torch.float64).to(self.dev)
        return t(case.X), t(case.Y), t(case.G)

    def inputs_for(self, case, X, Y, G):
        return make_inputs(X, Y, G, case.u_inf, case.v_inf, case.ub, case.vb, case.omega,
                           case.mode, case.gamma_b, case.znew, case.gamma_w,
                           getattr(case, "fbounds", ()))

    def outputs(self, nv: int, velocities=True) -> gpf_outputs:
        import torch
        if velocities and (self.u is None or self.u.numel() != nv):
            self.u = torch.empty(nv, dtype=torch.float64, device=self.dev)
            self.v = torch.empty(nv, dtype=torch.float64, device=self.dev)
        return make_outputs(self.psi, self.u if velocities else None,
                            self.v if velocities else None,
                            self.f if self.body else None, self.ftilde if self.body else None,
                            self.scalars, self.status)

    def solve(self, inp: gpf_inputs, X, stream=None, velocities=True):
        nv = int(X.numel()) if X is not None else 0
        out = self.outputs(nv, velocities)
        gpf_solve(self.plan, self.body, inp, out, stream)
        return out
