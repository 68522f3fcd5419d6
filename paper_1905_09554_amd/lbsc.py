"""ctypes binding of liblbsc.so (include/lbsc.h): argument marshalling only.

Every step of the method runs in the HIP kernels of the library; this module
allocates the device buffer through torch (memory and streams are torch's
job here), passes raw pointers and sizes, and turns status codes into
exceptions.  If the library has not been built, importing works but any
call raises: there is no CPU fallback.
"""
import ctypes
import os

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "liblbsc.so")

LBSC_OK = 0
LBSC_EINVAL = -1
LBSC_ENOMEM = -2
LBSC_EHIP = -3
LBSC_ENONFINITE = -4
LBSC_ESTATE = -5

BGK, MRT = 0, 1
FORCING_GUO, FORCING_SHIFT = 0, 1
F64, F32_SHIFTED = 0, 1

_COLL = {"bgk": BGK, "mrt": MRT}
_FORC = {"guo": FORCING_GUO, "shift": FORCING_SHIFT}
_PREC = {"f64": F64, "f32": F32_SHIFTED}


class Params(ctypes.Structure):
    _fields_ = [
        ("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32),
        ("collision", ctypes.c_int32), ("forcing", ctypes.c_int32), ("precision", ctypes.c_int32),
        ("G", ctypes.c_double), ("psi_rho0", ctypes.c_double), ("tau", ctypes.c_double),
        ("s_bulk", ctypes.c_double), ("s_ghost", ctypes.c_double), ("rho_ref", ctypes.c_double),
    ]


class Diag(ctypes.Structure):
    _fields_ = [
        ("mass", ctypes.c_double), ("mom", ctypes.c_double * 3), ("r_min", ctypes.c_double),
        ("z_argmin", ctypes.c_int32), ("reserved", ctypes.c_int32),
    ]


class Tuning(ctypes.Structure):
    _fields_ = [("threads", ctypes.c_int32), ("z_chunk", ctypes.c_int32),
                ("xcd_remap", ctypes.c_int32), ("block_y", ctypes.c_int32),
                ("pop_pad", ctypes.c_int32), ("nodes_per_thread", ctypes.c_int32),
                ("persistent", ctypes.c_int32), ("block_x", ctypes.c_int32),
                ("two_kernel", ctypes.c_int32)]


class LbscError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("lbsc error %d: %s" % (code, msg))
        self.code = code


_lib = None


def library():
    """Loads liblbsc.so once; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError("liblbsc.so is not built; run python -m paper_1905_09554_amd.build")
        lib = ctypes.CDLL(LIB_PATH)
        vp, i32, i64, dbl, sz = (ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64,
                                 ctypes.c_double, ctypes.c_size_t)
        P = ctypes.POINTER
        sig = {
            "lbsc_state_bytes": (sz, [P(Params)]),
            "lbsc_init_fields": (ctypes.c_int, [P(vp), P(Params), P(dbl), vp, sz, vp]),
            "lbsc_step": (ctypes.c_int, [vp, i64]),
            "lbsc_step_count": (i64, [vp]),
            "lbsc_compute_moments": (ctypes.c_int, [vp, vp, vp, vp]),
            "lbsc_interface_diagnostics": (ctypes.c_int, [vp, dbl, dbl, P(Diag), P(dbl)]),
            "lbsc_interface_diagnostics_static": (ctypes.c_int,
                                                  [vp, dbl, dbl, P(Diag), P(dbl)]),
            "lbsc_get_state": (ctypes.c_int, [vp, vp, sz, P(i64)]),
            "lbsc_set_state": (ctypes.c_int, [vp, vp, sz, i64]),
            "lbsc_set_tuning": (ctypes.c_int, [vp, P(Tuning)]),
            "lbsc_get_tuning": (ctypes.c_int, [vp, P(Tuning)]),
            "lbsc_default_tuning": (ctypes.c_int, [P(Params), i32, P(Tuning)]),
            "lbsc_lattice": (None, [P(i32), P(dbl)]),
            "lbsc_adjoint_workspace_bytes": (sz, [P(Params), i64, i32]),
            "lbsc_adjoint_forward": (ctypes.c_int, [vp, i64, i32, vp, sz]),
            "lbsc_rmin_gradient": (ctypes.c_int, [vp, dbl, dbl, vp, P(dbl)]),
            "lbsc_adjoint_backward": (ctypes.c_int, [vp, vp, vp, P(dbl), P(dbl)]),
            "lbsc_adjoint_rate_gradients": (ctypes.c_int, [vp, P(dbl), P(dbl)]),
            "lbsc_batch_state_bytes": (sz, [i32, P(Params)]),
            "lbsc_init_batch": (ctypes.c_int, [P(vp), i32, P(Params), P(P(dbl)), vp, sz, vp]),
            "lbsc_batch_size": (i32, [vp]),
            "lbsc_member_moments": (ctypes.c_int, [vp, i32, vp, vp, vp]),
            "lbsc_member_diagnostics": (ctypes.c_int, [vp, i32, dbl, dbl, P(Diag), P(dbl)]),
            "lbsc_member_get_state": (ctypes.c_int, [vp, i32, vp, sz]),
            "lbsc_member_set_state": (ctypes.c_int, [vp, i32, vp, sz]),
            "lbsc_destroy": (None, [vp]),
            "lbsc_last_error": (ctypes.c_char_p, [vp]),
        }
        for name, (res, args) in sig.items():
            fn = getattr(lib, name)
            fn.restype = res
            fn.argtypes = args
        _lib = lib
    return _lib


def make_params(nx, ny, nz, collision="bgk", forcing="guo", precision="f64", G=-5.0,
                tau=1.0, s_bulk=1.0, s_ghost=1.2, rho_ref=1.0, psi_rho0=1.0):
    return Params(nx, ny, nz, _COLL[collision], _FORC[forcing], _PREC[precision],
                  G, psi_rho0, tau, s_bulk, s_ghost, rho_ref)


def state_bytes(params):
    return library().lbsc_state_bytes(ctypes.byref(params))


def default_tuning(params):
    """The launch shape a context starts with (host only, no GPU): a dict
    like Simulation.get_tuning() for one Params, or a batch's for a list."""
    plist = list(params) if isinstance(params, (list, tuple)) else [params]
    arr = (Params * len(plist))(*plist)
    t = Tuning()
    _check(library().lbsc_default_tuning(arr, len(plist), ctypes.byref(t)))
    return {f: getattr(t, f) for f, _ in Tuning._fields_}


def lattice():
    """(c [19,3] int32, w [19] float64) in the library's population order."""
    c = np.zeros((19, 3), dtype=np.int32)
    w = np.zeros(19, dtype=np.float64)
    library().lbsc_lattice(c.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                           w.ctypes.data_as(ctypes.POINTER(ctypes.c_double)))
    return c, w


def _inputs_ready(device, stream):
    """The library's stream waits for torch's current stream, where device
    inputs (such as dL/drho) were made."""
    import torch
    cur = torch.cuda.current_stream(device)
    if cur != stream:
        stream.wait_stream(cur)


def _outputs_ready(device, stream, *tensors):
    """Torch's current stream waits for the library's stream, which wrote the
    device outputs; each output is also marked as used by that stream, so
    that torch's caching allocator does not hand its memory to other work
    before the stream is done with it."""
    import torch
    cur = torch.cuda.current_stream(device)
    if cur != stream:
        cur.wait_stream(stream)
        for t in tensors:
            if t is not None:
                t.record_stream(stream)


def _check(rc, ctx=None):
    if rc != LBSC_OK:
        msg = library().lbsc_last_error(ctx)
        raise LbscError(rc, msg.decode() if msg else "")


class Simulation:
    """One periodic box on one GPU.

    rho0: float64 array [nz, ny, nx] (host).  The device buffer is a torch
    uint8 tensor on ``device``; work goes to torch's current stream of that
    device unless ``stream`` (a torch.cuda.Stream) is given.  With a stream
    of its own, device tensors returned by a call are ordered after the
    library's work on torch's current stream, and device inputs made on
    torch's current stream before the call.
    """

    def __init__(self, rho0, params, device="cuda:0", stream=None):
        import torch
        self.params = params
        self.device = torch.device(device)
        rho0 = np.ascontiguousarray(rho0, dtype=np.float64)
        if rho0.shape != (params.nz, params.ny, params.nx):
            raise ValueError("rho0 shape %s != (nz, ny, nx)" % (rho0.shape,))
        nbytes = state_bytes(params)
        if nbytes == 0:
            raise LbscError(LBSC_EINVAL, "invalid parameters")
        self._buf = torch.empty(nbytes + 256, dtype=torch.uint8, device=self.device)
        base = self._buf.data_ptr()
        self._off = (-base) % 256
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        ctx = ctypes.c_void_p()
        rc = library().lbsc_init_fields(
            ctypes.byref(ctx), ctypes.byref(params),
            rho0.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
            ctypes.c_void_p(base + self._off), nbytes, ctypes.c_void_p(self.stream.cuda_stream))
        if rc != LBSC_OK:
            msg = library().lbsc_last_error(None)
            raise LbscError(rc, msg.decode() if msg else "")
        self._ctx = ctx
        self.n = params.nx * params.ny * params.nz
        self.elem = np.float64 if params.precision == F64 else np.float32

    # -- lifecycle
    def close(self):
        """Destroys the context and releases the device buffer (once the
        stream has finished with it)."""
        if getattr(self, "_ctx", None):
            library().lbsc_destroy(self._ctx)
            self._ctx = None
        if getattr(self, "_buf", None) is not None:
            self.stream.synchronize()
            self._buf = None
            self._ws = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- stepping
    def step(self, nsteps=1):
        _check(library().lbsc_step(self._ctx, int(nsteps)), self._ctx)

    @property
    def step_count(self):
        return int(library().lbsc_step_count(self._ctx))

    # -- outputs
    def moments(self, want_u=True, want_p=True):
        """(rho [nz,ny,nx], u^b [3,nz,ny,nx] or None, P or None) as float64 device tensors."""
        import torch
        p = self.params
        shape = (p.nz, p.ny, p.nx)
        rho = torch.empty(shape, dtype=torch.float64, device=self.device)
        u = torch.empty((3,) + shape, dtype=torch.float64, device=self.device) if want_u else None
        pr = torch.empty(shape, dtype=torch.float64, device=self.device) if want_p else None
        _check(library().lbsc_compute_moments(
            self._ctx, ctypes.c_void_p(rho.data_ptr()),
            ctypes.c_void_p(u.data_ptr() if u is not None else 0),
            ctypes.c_void_p(pr.data_ptr() if pr is not None else 0)), self._ctx)
        _outputs_ready(self.device, self.stream, rho, u, pr)
        return rho, u, pr

    def diagnostics(self, rho_v, rho_l):
        """dict(mass, mom, r_min, z_argmin, r_of_z) of the current state."""
        d = Diag()
        r = np.zeros(self.params.nz, dtype=np.float64)
        _check(library().lbsc_interface_diagnostics(
            self._ctx, float(rho_v), float(rho_l), ctypes.byref(d),
            r.ctypes.data_as(ctypes.POINTER(ctypes.c_double))), self._ctx)
        return {"mass": d.mass, "mom": [d.mom[0], d.mom[1], d.mom[2]], "r_min": d.r_min,
                "z_argmin": d.z_argmin, "r_of_z": r}

    # -- state
    def get_state(self):
        """Post-streaming populations [19, nz, ny, nx] in the storage precision."""
        p = self.params
        out = np.empty((19, p.nz, p.ny, p.nx), dtype=self.elem)
        step = ctypes.c_int64()
        _check(library().lbsc_get_state(self._ctx, ctypes.c_void_p(out.ctypes.data), out.nbytes,
                                        ctypes.byref(step)), self._ctx)
        return out, int(step.value)

    def set_state(self, pops, step=0):
        pops = np.ascontiguousarray(pops, dtype=self.elem)
        _check(library().lbsc_set_state(self._ctx, ctypes.c_void_p(pops.ctypes.data), pops.nbytes,
                                        int(step)), self._ctx)

    # -- adjoint
    def adjoint_forward(self, nsteps, segment):
        """Steps nsteps from the initial state saving checkpoints every
        `segment` steps in a device workspace owned by this object."""
        import torch
        nbytes = library().lbsc_adjoint_workspace_bytes(ctypes.byref(self.params), int(nsteps),
                                                        int(segment))
        if nbytes == 0:
            raise LbscError(LBSC_EINVAL, "invalid adjoint request")
        if getattr(self, "_ws", None) is not None:
            self.stream.synchronize()  # the old workspace may still be in use
            self._ws = None
        self._ws = torch.empty(nbytes + 256, dtype=torch.uint8, device=self.device)
        off = (-self._ws.data_ptr()) % 256
        _check(library().lbsc_adjoint_forward(self._ctx, int(nsteps), int(segment),
                                              ctypes.c_void_p(self._ws.data_ptr() + off), nbytes),
               self._ctx)

    def rmin_gradient(self, rho_v, rho_l):
        """(dr_min/drho as a float64 device tensor [nz,ny,nx], r_min)."""
        import torch
        p = self.params
        g = torch.empty((p.nz, p.ny, p.nx), dtype=torch.float64, device=self.device)
        r = ctypes.c_double()
        _check(library().lbsc_rmin_gradient(self._ctx, float(rho_v), float(rho_l),
                                            ctypes.c_void_p(g.data_ptr()), ctypes.byref(r)),
               self._ctx)
        _outputs_ready(self.device, self.stream, g)
        return g, r.value

    def adjoint_backward(self, rhobar):
        """(dL/drho0 device tensor, dL/dG, dL/dtau) for dL/drho_final = rhobar."""
        import torch
        rhobar = rhobar.to(device=self.device, dtype=torch.float64).contiguous()
        out = torch.empty_like(rhobar)
        _inputs_ready(self.device, self.stream)
        dG, dtau = ctypes.c_double(), ctypes.c_double()
        _check(library().lbsc_adjoint_backward(self._ctx, ctypes.c_void_p(rhobar.data_ptr()),
                                               ctypes.c_void_p(out.data_ptr()), ctypes.byref(dG),
                                               ctypes.byref(dtau)), self._ctx)
        _outputs_ready(self.device, self.stream, out, rhobar)
        return out, dG.value, dtau.value

    def rate_gradients(self):
        """(dL/ds_bulk, dL/ds_ghost) of the last adjoint_backward (MRT; 0 for BGK)."""
        b, g = ctypes.c_double(), ctypes.c_double()
        _check(library().lbsc_adjoint_rate_gradients(self._ctx, ctypes.byref(b),
                                                     ctypes.byref(g)), self._ctx)
        return b.value, g.value

    # -- launch shape
    def set_tuning(self, threads=0, z_chunk=0, xcd_remap=-1, block_y=0, pop_pad=-1,
                   nodes_per_thread=0, persistent=0, block_x=0, two_kernel=0):
        t = Tuning(threads, z_chunk, xcd_remap, block_y, pop_pad, nodes_per_thread, persistent,
                   block_x, two_kernel)
        _check(library().lbsc_set_tuning(self._ctx, ctypes.byref(t)), self._ctx)

    def get_tuning(self):
        t = Tuning()
        _check(library().lbsc_get_tuning(self._ctx, ctypes.byref(t)), self._ctx)
        return {"threads": t.threads, "z_chunk": t.z_chunk, "xcd_remap": t.xcd_remap,
                "block_y": t.block_y, "pop_pad": t.pop_pad,
                "nodes_per_thread": t.nodes_per_thread, "persistent": t.persistent,
                "block_x": t.block_x, "two_kernel": t.two_kernel}


class Batch:
    """Several periodic boxes stepped together on one GPU (one launch per
    step, or one cooperative launch for all steps with ``persistent=1``).

    rho0s: list of float64 arrays [nz, ny, nx]; params: list of Params with
    the same precision, collision and forcing.
    """

    def __init__(self, rho0s, params, device="cuda:0", stream=None):
        import torch
        if len(rho0s) != len(params) or not params:
            raise ValueError("need one rho0 per member")
        self.params = list(params)
        self.device = torch.device(device)
        self._rho = [np.ascontiguousarray(r, dtype=np.float64) for r in rho0s]
        for r, p in zip(self._rho, self.params):
            if r.shape != (p.nz, p.ny, p.nx):
                raise ValueError("rho0 shape %s != (nz, ny, nx)" % (r.shape,))
        n = len(params)
        parr = (Params * n)(*self.params)
        nbytes = library().lbsc_batch_state_bytes(n, parr)
        if nbytes == 0:
            raise LbscError(LBSC_EINVAL, "invalid batch parameters")
        self._buf = torch.empty(nbytes + 256, dtype=torch.uint8, device=self.device)
        base = self._buf.data_ptr()
        off = (-base) % 256
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        ptrs = (ctypes.POINTER(ctypes.c_double) * n)(
            *[r.ctypes.data_as(ctypes.POINTER(ctypes.c_double)) for r in self._rho])
        ctx = ctypes.c_void_p()
        rc = library().lbsc_init_batch(ctypes.byref(ctx), n, parr, ptrs,
                                       ctypes.c_void_p(base + off), nbytes,
                                       ctypes.c_void_p(self.stream.cuda_stream))
        if rc != LBSC_OK:
            msg = library().lbsc_last_error(None)
            raise LbscError(rc, msg.decode() if msg else "")
        self._ctx = ctx
        self.size = n

    def close(self):
        """Destroys the context and releases the device buffer (once the
        stream has finished with it)."""
        if getattr(self, "_ctx", None):
            library().lbsc_destroy(self._ctx)
            self._ctx = None
        if getattr(self, "_buf", None) is not None:
            self.stream.synchronize()
            self._buf = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def step(self, nsteps=1):
        _check(library().lbsc_step(self._ctx, int(nsteps)), self._ctx)

    @property
    def step_count(self):
        return int(library().lbsc_step_count(self._ctx))

    def set_tuning(self, **kw):
        Simulation.set_tuning(self, **kw)

    def get_tuning(self):
        return Simulation.get_tuning(self)

    def diagnostics(self, member, rho_v, rho_l):
        d = Diag()
        r = np.zeros(self.params[member].nz, dtype=np.float64)
        _check(library().lbsc_member_diagnostics(
            self._ctx, int(member), float(rho_v), float(rho_l), ctypes.byref(d),
            r.ctypes.data_as(ctypes.POINTER(ctypes.c_double))), self._ctx)
        return {"mass": d.mass, "mom": [d.mom[0], d.mom[1], d.mom[2]], "r_min": d.r_min,
                "z_argmin": d.z_argmin, "r_of_z": r}

    def moments(self, member, want_u=True, want_p=False):
        import torch
        p = self.params[member]
        shape = (p.nz, p.ny, p.nx)
        rho = torch.empty(shape, dtype=torch.float64, device=self.device)
        u = torch.empty((3,) + shape, dtype=torch.float64, device=self.device) if want_u else None
        pr = torch.empty(shape, dtype=torch.float64, device=self.device) if want_p else None
        _check(library().lbsc_member_moments(
            self._ctx, int(member), ctypes.c_void_p(rho.data_ptr()),
            ctypes.c_void_p(u.data_ptr() if u is not None else 0),
            ctypes.c_void_p(pr.data_ptr() if pr is not None else 0)), self._ctx)
        _outputs_ready(self.device, self.stream, rho, u, pr)
        return rho, u, pr

    def get_state(self, member):
        p = self.params[member]
        elem = np.float64 if p.precision == F64 else np.float32
        out = np.empty((19, p.nz, p.ny, p.nx), dtype=elem)
        _check(library().lbsc_member_get_state(self._ctx, int(member),
                                               ctypes.c_void_p(out.ctypes.data), out.nbytes),
               self._ctx)
        return out
