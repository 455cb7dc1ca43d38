"""ctypes binding of librts (include/rts.h): argument marshalling only.

Every step of the solve runs in the gfx950 kernels of `librts.so`; this
module converts problem descriptions into the C structs, passes device
pointers of torch tensors and the current HIP stream, and turns non-zero
status codes into exceptions.  There is no fallback: if the library is not
built, importing works but every call raises.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "librts.so")

RTS_OK = 0
RTS_E_ARG = -1
RTS_E_UNSUPPORTED = -2
RTS_E_WORKSPACE = -3
RTS_E_HIP = -4
RTS_E_DEADLOCK = -5
RTS_E_NOT_BUILT = -6
RTS_E_NONFINITE = -7
RTS_FP64 = 0
RTS_FP32 = 1
RTS_OP_SOLVE = 0
RTS_OP_ADJOINT = 1
RTS_OP_AUTOTUNE = 2

# every symbol declared in include/rts.h
SYMBOLS = ("rts_plan_create", "rts_workspace_bytes", "rts_solve", "rts_solve_batched",
           "rts_adjoint", "rts_solve_for_adjoint", "rts_adjoint_from_solve", "rts_plan_autotune",
           "rts_check_status", "rts_plan_get_schedule", "rts_plan_set_schedule",
           "rts_plan_enable_timing", "rts_plan_last_timing",
           "rts_plan_destroy", "rts_status_string", "rts_version", "rts_solve_static",
           "rts_check_inputs")
# rts_solve_static's fixed device array (bytes)
RTS_STATIC_SCRATCH_BYTES = 64 << 20


class Grid(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32),
                ("dx", ctypes.c_double), ("dy", ctypes.c_double), ("dz", ctypes.c_double)]


class Desc(ctypes.Structure):
    _fields_ = [("g", Grid), ("nbands", ctypes.c_int32), ("nrays", ctypes.c_int32),
                ("mu", ctypes.POINTER(ctypes.c_double)), ("w", ctypes.POINTER(ctypes.c_double)),
                ("qweight", ctypes.POINTER(ctypes.c_double)), ("bot", ctypes.c_int32),
                ("top", ctypes.c_int32), ("i_bot", ctypes.c_double), ("n_iter", ctypes.c_int32),
                ("prec", ctypes.c_int32), ("flux", ctypes.c_int32), ("tol", ctypes.c_double),
                ("sub", ctypes.c_int32 * 3), ("gs_iter", ctypes.c_int32)]


class Inputs(ctypes.Structure):
    _fields_ = [("kappa", ctypes.c_void_p), ("rho", ctypes.c_void_p), ("S", ctypes.c_void_p),
                ("eps", ctypes.c_void_p), ("ghost", ctypes.c_void_p)]


class Outputs(ctypes.Structure):
    _fields_ = [("Q", ctypes.c_void_p), ("J", ctypes.c_void_p), ("I_top", ctypes.c_void_p),
                ("F", ctypes.c_void_p), ("QF", ctypes.c_void_p), ("S", ctypes.c_void_p),
                ("ghost", ctypes.c_void_p)]


def _ptr_or_none(t):
    return t.data_ptr() if t is not None else None


def _marshal(ins, outs):
    """C arrays of rts_inputs / rts_outputs; ins entries are (kappa, rho, S[, eps[, ghost]]);
    outs entries are (Q, J, I_top[, F, QF[, S[, ghost]]]); any but Q and the inputs may be
    None."""
    n = len(ins)
    ci = (Inputs * n)()
    co = (Outputs * n)()
    for i, (inp, o) in enumerate(zip(ins, outs)):
        inp = tuple(inp) + (None,) * (5 - len(inp))
        ci[i] = Inputs(*(_ptr_or_none(t) for t in inp))
        o = tuple(o) + (None,) * (7 - len(o))
        co[i] = Outputs(*(_ptr_or_none(t) for t in o))
    return ci, co


class Seeds(ctypes.Structure):
    _fields_ = [("gQ", ctypes.c_void_p), ("gJ", ctypes.c_void_p), ("gItop", ctypes.c_void_p)]


class Grads(ctypes.Structure):
    _fields_ = [("dS", ctypes.c_void_p), ("dchi", ctypes.c_void_p)]


class Schedule(ctypes.Structure):
    _fields_ = [("rows_per_strip", ctypes.c_int32), ("max_workgroups", ctypes.c_int32),
                ("order", ctypes.c_int32), ("use_graph", ctypes.c_int32),
                ("single_launch", ctypes.c_int32), ("split_reverse", ctypes.c_int32)]


class RTSError(RuntimeError):
    def __init__(self, status: int, where: str):
        self.status = status
        super().__init__(f"{where}: {status_string(status)}")


_lib = None


def lib():
    """The loaded librts (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"librts.so not built ({LIB_PATH}); run __graft_entry__.build()")
        try:
            # torch ships its own HIP runtime under the same soname: loaded first, it is the
            # one librts binds to (loaded after librts, it would be a second runtime in the
            # process and find no GPU)
            import torch  # noqa: F401
        except ImportError:
            pass
        L = ctypes.CDLL(LIB_PATH)
        vp, i32, sz = ctypes.c_void_p, ctypes.c_int32, ctypes.c_size_t
        L.rts_plan_create.argtypes = [ctypes.POINTER(Desc), i32, ctypes.POINTER(vp)]
        L.rts_workspace_bytes.argtypes = [vp, i32, ctypes.POINTER(sz)]
        L.rts_solve.argtypes = [vp, ctypes.POINTER(Inputs), ctypes.POINTER(Outputs), vp, sz, vp]
        L.rts_solve_batched.argtypes = [vp, i32, ctypes.POINTER(Inputs), ctypes.POINTER(Outputs),
                                        vp, sz, vp]
        L.rts_adjoint.argtypes = [vp, i32, ctypes.POINTER(Inputs), ctypes.POINTER(Seeds),
                                  ctypes.POINTER(Grads), vp, sz, vp]
        L.rts_adjoint_from_solve.argtypes = L.rts_adjoint.argtypes
        L.rts_solve_for_adjoint.argtypes = [vp, i32, ctypes.POINTER(Inputs),
                                            ctypes.POINTER(Outputs), vp, sz, vp]
        L.rts_solve_static.argtypes = [vp, i32, ctypes.POINTER(Inputs), ctypes.POINTER(Outputs),
                                       vp]
        L.rts_plan_autotune.argtypes = [vp, i32, ctypes.POINTER(Inputs), ctypes.POINTER(Outputs),
                                         vp, sz, vp, i32, ctypes.POINTER(Schedule)]
        L.rts_check_status.argtypes = [vp, vp, vp]
        L.rts_check_inputs.argtypes = [vp, i32, ctypes.POINTER(Inputs), vp, sz, vp]
        L.rts_plan_get_schedule.argtypes = [vp, ctypes.POINTER(Schedule)]
        L.rts_plan_set_schedule.argtypes = [vp, ctypes.POINTER(Schedule)]
        L.rts_plan_enable_timing.argtypes = [vp, i32]
        L.rts_plan_last_timing.argtypes = [vp, ctypes.POINTER(ctypes.c_double),
                                           ctypes.POINTER(ctypes.c_double)]
        L.rts_plan_destroy.argtypes = [vp]
        L.rts_plan_destroy.restype = None
        L.rts_status_string.argtypes = [ctypes.c_int]
        L.rts_status_string.restype = ctypes.c_char_p
        L.rts_version.argtypes = []
        L.rts_version.restype = ctypes.c_char_p
        for f in ("rts_plan_create", "rts_workspace_bytes", "rts_solve", "rts_solve_batched",
                  "rts_adjoint", "rts_solve_for_adjoint", "rts_adjoint_from_solve",
                  "rts_plan_autotune", "rts_check_status", "rts_plan_get_schedule", "rts_solve_static",
                  "rts_check_inputs",
                  "rts_plan_set_schedule", "rts_plan_enable_timing", "rts_plan_last_timing"):
            getattr(L, f).restype = ctypes.c_int
        _lib = L
    return _lib


def status_string(status: int) -> str:
    return lib().rts_status_string(int(status)).decode()


def _check(status: int, where: str):
    if status != RTS_OK:
        raise RTSError(status, where)


def _stream_ptr(stream=None):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


class Plan:
    """A librts plan for one or more boxes (paper_2107_08145_amd.inputs.Problem)."""

    def __init__(self, problems, prec: int = RTS_FP64, flux=False, tol: float = 0.0, sub=None,
                 gs_iter: int = 0):
        """flux: bool, or one bool per box (desc.flux: room for the flux vector);
        tol: desc.tol of every box (0: n_iter sweeps; > 0: tolerance-driven);
        sub: desc.sub, (mx, my, mz) subdomains with lagged exchange, or None (undivided),
        for every box, or a list with one such entry per box."""
        if not isinstance(problems, (list, tuple)):
            problems = [problems]
        flags = list(flux) if isinstance(flux, (list, tuple)) else [flux] * len(problems)
        self.problems = list(problems)
        self.prec = prec
        self._keep = []
        descs = (Desc * len(problems))()
        for i, p in enumerate(problems):
            mu = np.ascontiguousarray(p.mu, dtype=np.float64)
            w = np.ascontiguousarray(p.w, dtype=np.float64)
            qw = np.ascontiguousarray(p.qweight, dtype=np.float64)
            self._keep += [mu, w, qw]
            d = descs[i]
            d.g = Grid(p.nx, p.ny, p.nz, p.dx, p.dy, p.dz)
            d.nbands, d.nrays = p.nbands, p.nrays
            d.mu = mu.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
            d.w = w.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
            d.qweight = qw.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
            d.bot, d.top, d.i_bot, d.n_iter, d.prec = p.bot, p.top, p.i_bot, p.n_iter, prec
            d.flux = 1 if flags[i] else 0
            d.tol = float(tol)
            d.gs_iter = int(gs_iter)
            sb = sub[i] if isinstance(sub, list) else sub
            if sb is not None:
                d.sub[0], d.sub[1], d.sub[2] = (int(v) for v in sb)
        h = ctypes.c_void_p()
        _check(lib().rts_plan_create(descs, len(problems), ctypes.byref(h)), "rts_plan_create")
        self.handle = h
        self._ws = None

    def __del__(self):
        h = getattr(self, "handle", None)
        if h is not None and h.value and _lib is not None:
            _lib.rts_plan_destroy(h)
            self.handle = None

    def workspace_bytes(self, op: int = RTS_OP_SOLVE) -> int:
        n = ctypes.c_size_t()
        _check(lib().rts_workspace_bytes(self.handle, op, ctypes.byref(n)), "rts_workspace_bytes")
        return n.value

    def schedule(self) -> dict:
        s = Schedule()
        _check(lib().rts_plan_get_schedule(self.handle, ctypes.byref(s)), "rts_plan_get_schedule")
        return {k: getattr(s, k) for k, _ in Schedule._fields_}

    def set_schedule(self, **kw):
        cur = self.schedule()
        cur.update(kw)
        s = Schedule(**cur)
        _check(lib().rts_plan_set_schedule(self.handle, ctypes.byref(s)), "rts_plan_set_schedule")
        self._ws = None

    def enable_timing(self, on: bool = True):
        _check(lib().rts_plan_enable_timing(self.handle, 1 if on else 0), "rts_plan_enable_timing")

    def last_timing(self):
        a, b = ctypes.c_double(), ctypes.c_double()
        _check(lib().rts_plan_last_timing(self.handle, ctypes.byref(a), ctypes.byref(b)),
               "rts_plan_last_timing")
        return a.value, b.value

    def release_workspace(self):
        """Drop the plan's own workspace (the next call allocates one again)."""
        self._ws = None

    def workspace(self, op: int = RTS_OP_SOLVE):
        import torch
        need = self.workspace_bytes(op)
        if self._ws is None or self._ws.numel() < need:
            self._ws = torch.empty(need + 256, dtype=torch.uint8, device="cuda")
        base = self._ws.data_ptr()
        off = (-base) % 256
        return base + off, self._ws.numel() - off

    # -- device arrays -------------------------------------------------------
    @property
    def dtype(self):
        import torch
        return torch.float32 if self.prec == RTS_FP32 else torch.float64

    def device_inputs(self, p):
        import torch
        dt = self.dtype
        return (torch.as_tensor(np.ascontiguousarray(p.kappa)).to("cuda", dt).contiguous(),
                torch.as_tensor(np.ascontiguousarray(p.rho)).to("cuda", dt).contiguous(),
                torch.as_tensor(np.ascontiguousarray(p.S)).to("cuda", dt).contiguous())

    def new_outputs(self, p, want_j=True, want_itop=True, want_flux=False):
        """(Q, J, I_top), or (Q, J, I_top, F, QF) with want_flux (F [3,nz,ny,nx], QF
        [nz,ny,nx], float64)."""
        import torch
        Q = torch.empty((p.nz, p.ny, p.nx), dtype=torch.float64, device="cuda")
        J = torch.empty((p.nbands, p.nz, p.ny, p.nx), dtype=self.dtype, device="cuda") if want_j else None
        It = (torch.empty((p.nbands, p.n_up, p.ny, p.nx), dtype=self.dtype, device="cuda")
              if want_itop else None)
        if not want_flux:
            return Q, J, It
        F = torch.empty((3, p.nz, p.ny, p.nx), dtype=torch.float64, device="cuda")
        QF = torch.empty((p.nz, p.ny, p.nx), dtype=torch.float64, device="cuda")
        return Q, J, It, F, QF

    def solve_into(self, ins, outs, stream=None, batched=False):
        """Enqueue a forward solve.  ins: [(kappa, rho, S)] per box; outs: [(Q, J, I_top)] or
        [(Q, J, I_top, F, QF)] per box."""
        n = len(ins)
        ci, co = _marshal(ins, outs)
        ws, nbytes = self.workspace()
        st = _stream_ptr(stream)
        if batched:
            rc = lib().rts_solve_batched(self.handle, n, ci, co, ctypes.c_void_p(ws), nbytes, st)
        else:
            rc = lib().rts_solve(self.handle, ci, co, ctypes.c_void_p(ws), nbytes, st)
        _check(rc, "rts_solve_batched" if batched else "rts_solve")

    def solve_static_into(self, ins, outs, stream=None):
        """rts_solve_static: the forward solve of all boxes on the library's fixed device
        array (no workspace, nothing allocated)."""
        ci, co = _marshal(ins, outs)
        _check(lib().rts_solve_static(self.handle, len(ins), ci, co, _stream_ptr(stream)),
               "rts_solve_static")

    def check_static_status(self, stream=None):
        """Synchronise and read the status word rts_solve_static left on this device."""
        _check(lib().rts_check_status(self.handle, None, _stream_ptr(stream)), "device status")

    def autotune(self, ins, outs, reps: int = 3, stream=None) -> dict:
        """Time every candidate schedule on these inputs (rts_plan_autotune) and keep
        the fastest; returns it."""
        n = len(ins)
        ci, co = _marshal(ins, outs)
        ws, nbytes = self.workspace(RTS_OP_AUTOTUNE)
        sch = Schedule()
        _check(lib().rts_plan_autotune(self.handle, n, ci, co, ctypes.c_void_p(ws), nbytes,
                                       _stream_ptr(stream), reps, ctypes.byref(sch)),
               "rts_plan_autotune")
        return {k: getattr(sch, k) for k, _ in Schedule._fields_}

    def adjoint_workspace(self):
        """A private adjoint workspace: (tensor, aligned pointer, bytes)."""
        import torch
        need = self.workspace_bytes(RTS_OP_ADJOINT)
        t = torch.empty(need + 256, dtype=torch.uint8, device="cuda")
        off = (-t.data_ptr()) % 256
        return t, t.data_ptr() + off, t.numel() - off

    def solve_for_adjoint_into(self, ins, outs, ws=None, stream=None):
        """rts_solve_for_adjoint: the forward solve that also keeps D of every plane for
        adjoint_from_solve_into; ws = (pointer, bytes) of an adjoint workspace (default: the
        plan's own)."""
        n = len(ins)
        ci, co = _marshal(ins, outs)
        w, nbytes = ws if ws is not None else self.workspace(RTS_OP_ADJOINT)
        _check(lib().rts_solve_for_adjoint(self.handle, n, ci, co, ctypes.c_void_p(w), nbytes,
                                           _stream_ptr(stream)), "rts_solve_for_adjoint")

    def adjoint_from_solve_into(self, ins, seeds, grads, ws=None, stream=None):
        """rts_adjoint_from_solve on the workspace of the last solve_for_adjoint_into."""
        n = len(ins)
        ci = (Inputs * n)()
        cs = (Seeds * n)()
        cg = (Grads * n)()
        ptr = (lambda t: t.data_ptr() if t is not None else None)
        for i, ((k, r, s), (gq, gj, gi), (ds, dc)) in enumerate(zip(ins, seeds, grads)):
            ci[i] = Inputs(k.data_ptr(), r.data_ptr(), s.data_ptr())
            cs[i] = Seeds(ptr(gq), ptr(gj), ptr(gi))
            cg[i] = Grads(ds.data_ptr(), dc.data_ptr())
        w, nbytes = ws if ws is not None else self.workspace(RTS_OP_ADJOINT)
        _check(lib().rts_adjoint_from_solve(self.handle, n, ci, cs, cg, ctypes.c_void_p(w), nbytes,
                                            _stream_ptr(stream)), "rts_adjoint_from_solve")

    def adjoint_into(self, ins, seeds, grads, stream=None):
        """Enqueue an adjoint.  ins: [(kappa, rho, S)]; seeds: [(gQ, gJ, gItop)] (any may be
        None); grads: [(dS, dchi)] per box."""
        n = len(ins)
        ci = (Inputs * n)()
        cs = (Seeds * n)()
        cg = (Grads * n)()
        ptr = (lambda t: t.data_ptr() if t is not None else None)
        for i, ((k, r, s), (gq, gj, gi), (ds, dc)) in enumerate(zip(ins, seeds, grads)):
            ci[i] = Inputs(k.data_ptr(), r.data_ptr(), s.data_ptr())
            cs[i] = Seeds(ptr(gq), ptr(gj), ptr(gi))
            cg[i] = Grads(ds.data_ptr(), dc.data_ptr())
        ws, nbytes = self.workspace(RTS_OP_ADJOINT)
        _check(lib().rts_adjoint(self.handle, n, ci, cs, cg, ctypes.c_void_p(ws), nbytes,
                                 _stream_ptr(stream)), "rts_adjoint")

    def check_inputs(self, ins, stream=None):
        """rts_check_inputs: raise RTSError(RTS_E_NONFINITE) if any box's kappa, rho, S (or
        eps) holds a NaN or an infinity; uses the plan's own workspace."""
        n = len(ins)
        ci, _ = _marshal(ins, [(None,)] * n)
        ws, nbytes = self.workspace()
        _check(lib().rts_check_inputs(self.handle, n, ci, ctypes.c_void_p(ws), nbytes,
                                      _stream_ptr(stream)), "rts_check_inputs")

    def check_status(self, stream=None, ws=None):
        """rts_check_status: synchronise the stream and raise RTSError if the last call on the
        workspace (default: the plan's own; else a pointer, or (pointer, bytes)) left an error
        in its status word (RTS_E_DEADLOCK)."""
        if ws is None:
            ws, _ = self.workspace()
        elif isinstance(ws, tuple):
            ws = ws[0]
        _check(lib().rts_check_status(self.handle, ctypes.c_void_p(ws), _stream_ptr(stream)),
               "rts_check_status")


def solve(p, prec: int = RTS_FP64, plan: Plan | None = None, flux: bool = False,
          tol: float = 0.0, sub=None):
    """Forward solve of one problem on the current GPU; returns numpy (Q, J, I_top), or
    (Q, J, I_top, F, QF) with flux; tol > 0: tolerance-driven boundary iteration; sub:
    (mx, my, mz) subdomains with lagged exchange."""
    import torch
    plan = plan or Plan(p, prec, flux=flux, tol=tol, sub=sub)
    ins = plan.device_inputs(p)
    outs = plan.new_outputs(p, want_flux=flux)
    plan.solve_into([ins], [outs])
    plan.check_status()
    torch.cuda.synchronize()
    return tuple(o.double().cpu().numpy() for o in outs)


def solve_warm(p, prec: int, ghost_in=None, tol: float = 0.0, plan: Plan | None = None):
    """Forward solve from given initial ghost planes (rts_inputs.ghost, warm start;
    None: cold) that also returns the final ghost planes: numpy (Q, J, I_top, ghost_out),
    ghost arrays [B, R, nz, max(nx, ny)] in the plan's precision."""
    import torch
    plan = plan or Plan(p, prec, tol=tol)
    k, r, s = plan.device_inputs(p)
    shape = (p.nbands, p.nrays, p.nz, max(p.nx, p.ny))
    gi = None if ghost_in is None else torch.as_tensor(
        np.ascontiguousarray(ghost_in)).to("cuda", plan.dtype).contiguous()
    go = torch.zeros(shape, dtype=plan.dtype, device="cuda")
    Q, J, It = plan.new_outputs(p)
    plan.solve_into([(k, r, s, None, gi)], [(Q, J, It, None, None, None, go)])
    plan.check_status()
    torch.cuda.synchronize()
    return tuple(o.double().cpu().numpy() for o in (Q, J, It, go))


def solve_gs(p, eps, gs_iter: int, plan: Plan | None = None):
    """Scattering solve (desc.gs_iter > 0, FP64) of one problem on the current GPU:
    p.S is the thermal source B, eps [B,nz,ny,nx] the photon destruction
    probability.  Returns numpy (Q, J, I_top, S)."""
    import torch
    plan = plan or Plan(p, RTS_FP64, gs_iter=gs_iter)
    k, r, s = plan.device_inputs(p)
    e = torch.as_tensor(np.ascontiguousarray(eps, dtype=np.float64)).to("cuda")
    Q, J, It = plan.new_outputs(p)
    S = torch.empty_like(J)
    plan.solve_into([(k, r, s, e)], [(Q, J, It, None, None, S)])
    plan.check_status()
    torch.cuda.synchronize()
    return tuple(o.double().cpu().numpy() for o in (Q, J, It, S))


def adjoint(p, prec: int = RTS_FP64, gQ=None, gJ=None, gItop=None, plan: Plan | None = None):
    """Gradients (dL/dS, dL/dchi) as numpy [B,nz,ny,nx] of L = <gQ,Q> + <gJ,J> + <gItop,I_top>
    for one problem on the current GPU."""
    import torch
    plan = plan or Plan(p, prec)
    ins = plan.device_inputs(p)
    dev = (lambda a, dt: None if a is None else
           torch.as_tensor(np.ascontiguousarray(a)).to("cuda", dt).contiguous())
    seeds = (dev(gQ, torch.float64), dev(gJ, plan.dtype), dev(gItop, plan.dtype))
    dS = torch.empty((p.nbands, p.nz, p.ny, p.nx), dtype=plan.dtype, device="cuda")
    dchi = torch.empty_like(dS)
    plan.adjoint_into([ins], [seeds], [(dS, dchi)])
    plan.check_status()
    torch.cuda.synchronize()
    return dS.double().cpu().numpy(), dchi.double().cpu().numpy()
