"""ctypes binding of libsem.so (include/sem.h).

Argument marshalling only: every numerical step runs in the library's HIP
kernels.  PyTorch provides device memory (the workspace and the I/O tensors)
and the stream.  Importing this module loads the shared library and raises
if it is missing: there is no CPU fallback.
"""
import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIBPATH = os.path.join(HERE, "libsem.so")

# The library must share PyTorch's HIP runtime (streams and allocations come
# from torch): load torch first so that its libamdhip64 satisfies libsem.so's
# dependency instead of a second runtime instance.
import torch  # noqa: E402,F401

if not os.path.exists(LIBPATH):
    raise ImportError(f"{LIBPATH} is missing: build it with `python -m paper_1512_02548_amd.build` "
                      "(there is no CPU fallback)")
_lib = C.CDLL(LIBPATH)

SEM_OK, SEM_E_INVAL, SEM_E_NOMEM, SEM_E_DOMAIN, SEM_E_NOCONV, SEM_E_BREAKDOWN, SEM_E_NONFINITE, SEM_E_DEVICE = range(8)
STATUS_NAMES = {0: "OK", 1: "INVAL", 2: "NOMEM", 3: "DOMAIN", 4: "NOCONV", 5: "BREAKDOWN", 6: "NONFINITE",
                7: "DEVICE"}
SEM_PREC_FP64, SEM_PREC_FP32_IR, SEM_PREC_BF16_IR = 0, 1, 2
SEM_RECOVER_DX, SEM_RECOVER_W = 0, 1
SEM_OP_STIFFNESS, SEM_OP_MASS2D, SEM_OP_PRECOND, SEM_OP_SZ = 0, 1, 2, 3


class sem_mesh_desc(C.Structure):
    _fields_ = [("nx", C.c_int32), ("nz", C.c_int32), ("order", C.c_int32), ("periodic", C.c_int32),
                ("length", C.c_double), ("g", C.c_double),
                ("h", C.POINTER(C.c_double)), ("h_x", C.POINTER(C.c_double)),
                ("sigma_levels", C.POINTER(C.c_double)),
                ("filter_ic", C.c_int32), ("filter_sigma", C.c_double),
                ("overint_order", C.c_int32), ("restart", C.c_int32), ("variant", C.c_int32),
                ("tiles_per_block", C.c_int32)]


class sem_mesh_info(C.Structure):
    _fields_ = [("n", C.c_int64), ("ns", C.c_int64), ("n_free", C.c_int64), ("n_elem", C.c_int64),
                ("np", C.c_int32), ("nblocks", C.c_int32), ("workspace_bytes", C.c_uint64)]


class sem_solve_opts(C.Structure):
    _fields_ = [("rtol", C.c_double), ("max_iter", C.c_int32), ("prec", C.c_int32),
                ("inner_rtol", C.c_double), ("max_refine", C.c_int32), ("warm_start", C.c_int32),
                ("lookahead", C.c_int32), ("predict", C.c_int32)]


class sem_solve_stats(C.Structure):
    _fields_ = [("iters", C.c_int32), ("refinements", C.c_int32), ("rel_residual", C.c_double),
                ("seconds", C.c_double), ("status", C.c_int32), ("reserved", C.c_int32)]

    def as_dict(self):
        return dict(iters=self.iters, refinements=self.refinements, rel_residual=self.rel_residual,
                    seconds=self.seconds, status=self.status)


_P = C.c_void_p
_D = C.POINTER(C.c_double)
_SIGS = {
    "sem_mesh_create": (C.c_int, [C.POINTER(sem_mesh_desc), C.POINTER(_P)]),
    "sem_mesh_query": (C.c_int, [_P, C.POINTER(sem_mesh_info)]),
    "sem_mesh_bind": (C.c_int, [_P, _P, C.c_size_t, _P]),
    "sem_mesh_node_coords": (C.c_int, [_P, _D, _D]),
    "sem_mesh_surface_nodes": (C.c_int, [_P, C.POINTER(C.c_int64)]),
    "sem_mesh_destroy": (None, [_P]),
    "sem_reference_operators": (C.c_int, [C.c_int32, C.c_int32, C.c_int32, C.c_double] + [_D] * 8),
    "sem_set_surface": (C.c_int, [_P, _P, _P, _P]),
    "sem_apply": (C.c_int, [_P, C.c_int, _P, _P, _P]),
    "sem_apply_timed": (C.c_int, [_P, C.c_int, C.c_int32, _P, _P, C.c_int32, C.POINTER(C.c_float), _P]),
    "sem_laplace_solve": (C.c_int, [_P, _P, _P, _P, _P, C.POINTER(sem_solve_opts),
                                    C.POINTER(sem_solve_stats), _P]),
    "sem_gradient_recover": (C.c_int, [_P, C.c_int, _P, _P, _P, _P]),
    "sem_recover_kinematics": (C.c_int, [_P, _P, _P, _P, _P, _P, _P]),
    "sem_free_surface_rhs": (C.c_int, [_P, _P, _P, _P, _P, _P, _P, _P]),
    "sem_free_surface_rhs_noalloc": (C.c_int, [_P, _P, _P, _P, _P, _P, _P, _P]),
    "sem_rk4_step": (C.c_int, [_P, _P, _P, _P, C.c_double, C.POINTER(sem_solve_opts),
                               C.POINTER(sem_solve_stats), _P]),
    "sem_rk4_reset_history": (C.c_int, [_P, _P]),
    "sem_set_relaxation": (C.c_int, [_P, _D]),
    "sem_rk4_step_forced": (C.c_int, [_P, _P, _P, _P, C.c_double, _P, C.POINTER(sem_solve_opts),
                                      C.POINTER(sem_solve_stats), _P]),
    "sem_batch_create": (C.c_int, [C.POINTER(_P), C.c_int32, C.c_int32, _P, C.POINTER(_P)]),
    "sem_batch_laplace_solve": (C.c_int, [_P, C.POINTER(_P), C.POINTER(_P), C.POINTER(_P), C.POINTER(_P),
                                          C.POINTER(C.c_uint8), C.POINTER(sem_solve_opts),
                                          C.POINTER(C.c_int32), C.POINTER(C.c_int32), _P]),
    "sem_batch_rk4_step": (C.c_int, [_P, C.POINTER(_P), C.POINTER(_P), C.POINTER(_P), _D,
                                     C.POINTER(C.c_uint8), C.POINTER(sem_solve_opts),
                                     C.POINTER(C.c_int32), C.POINTER(C.c_int32), _P]),
    "sem_batch_destroy": (None, [_P]),
    "sem_batch_apply_timed": (C.c_int, [_P, C.c_int32, C.c_int32, C.c_int32, C.POINTER(C.c_float), _P]),
    "sem_batch_graphs": (C.c_int, [_P, C.c_int32]),
    "sem_batch_graph_count": (C.c_int, [_P, C.POINTER(C.c_int32)]),
    "sem_selftest_mfma": (C.c_int, [_P, C.POINTER(C.c_double), _D, _P]),
    "sem_kernel_timing": (C.c_int, [_P, C.c_int32]),
    "sem_kernel_timing_read": (C.c_int, [_P, C.POINTER(C.c_int64), C.POINTER(C.c_double)]),
    "sem_last_error": (C.c_char_p, []),
}
for _name, (_res, _args) in _SIGS.items():
    _f = getattr(_lib, _name)
    _f.restype = _res
    _f.argtypes = _args
    globals()[_name] = _f


class SemError(RuntimeError):
    def __init__(self, code, where):
        self.code = code
        msg = sem_last_error()
        super().__init__(f"{where}: {STATUS_NAMES.get(code, code)} ({msg.decode() if msg else ''})")


def check(code, where):
    if code != SEM_OK:
        raise SemError(code, where)


def _ptr(t):
    return C.c_void_p(t.data_ptr())


def _stream(stream=None):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return C.c_void_p(s.cuda_stream)


def default_opts(rtol=1e-12, max_iter=5000, prec=SEM_PREC_FP64, inner_rtol=1e-4, max_refine=30,
                 warm_start=0, lookahead=2, predict=5):
    return sem_solve_opts(rtol, max_iter, prec, inner_rtol, max_refine, warm_start, lookahead, predict)


class Mesh:
    """A tank on the device: mesh_create + query + a torch-allocated workspace + bind."""

    def __init__(self, nx, nz, P, length, periodic, h, hx, g=9.81, sigma_levels=None, filter_ic=None,
                 filter_sigma=1.0, overint=None, restart=30, variant=0, tiles_per_block=0, device="cuda", bind=True):
        self.h = np.ascontiguousarray(h, dtype=np.float64)
        self.hx = np.ascontiguousarray(hx, dtype=np.float64)
        self._sl = None if sigma_levels is None else np.ascontiguousarray(sigma_levels, dtype=np.float64)
        dp = lambda a: a.ctypes.data_as(_D) if a is not None else None
        desc = sem_mesh_desc(nx, nz, P, 1 if periodic else 0, float(length), float(g), dp(self.h), dp(self.hx),
                             dp(self._sl), P + 1 if filter_ic is None else filter_ic, float(filter_sigma),
                             P if overint is None else overint, restart, variant, int(tiles_per_block))
        self.handle = C.c_void_p()
        check(sem_mesh_create(C.byref(desc), C.byref(self.handle)), "sem_mesh_create")
        self.info = sem_mesh_info()
        check(sem_mesh_query(self.handle, C.byref(self.info)), "sem_mesh_query")
        self.n, self.ns = self.info.n, self.info.ns
        self.workspace = None
        if bind:
            self.bind(device)

    def bind(self, device="cuda"):
        import torch
        nbytes = int(self.info.workspace_bytes)
        self.workspace = torch.empty(nbytes + 256, dtype=torch.uint8, device=device)
        off = (-self.workspace.data_ptr()) % 256
        ptr = C.c_void_p(self.workspace.data_ptr() + off)
        check(sem_mesh_bind(self.handle, ptr, nbytes, _stream()), "sem_mesh_bind")

    def node_coords(self):
        x = np.empty(self.n)
        s = np.empty(self.n)
        check(sem_mesh_node_coords(self.handle, x.ctypes.data_as(_D), s.ctypes.data_as(_D)), "node_coords")
        return x, s

    def surface_nodes(self):
        idx = np.empty(self.ns, dtype=np.int64)
        check(sem_mesh_surface_nodes(self.handle, idx.ctypes.data_as(C.POINTER(C.c_int64))), "surface_nodes")
        return idx

    def surface_x(self):
        x, _ = self.node_coords()
        return x[self.surface_nodes()]

    # --- device calls (tensors are float64, contiguous, on the GPU)
    def set_surface(self, eta, etax, stream=None):
        check(sem_set_surface(self.handle, _ptr(eta), _ptr(etax), _stream(stream)), "sem_set_surface")

    def apply(self, op, u, y, stream=None):
        check(sem_apply(self.handle, op, _ptr(u), _ptr(y), _stream(stream)), "sem_apply")

    def selftest_mfma(self, raw=False, stream=None):
        err = C.c_double()
        buf = np.zeros(512)
        check(sem_selftest_mfma(self.handle, C.byref(err), buf.ctypes.data_as(_D), _stream(stream)),
              "sem_selftest_mfma")
        return (err.value, buf) if raw else err.value

    def apply_timed(self, op, u, y, reps, prec=SEM_PREC_FP64, stream=None):
        ms = C.c_float()
        check(sem_apply_timed(self.handle, op, prec, _ptr(u), _ptr(y), int(reps), C.byref(ms), _stream(stream)),
              "sem_apply_timed")
        return ms.value

    def kernel_timing(self, enable):
        check(sem_kernel_timing(self.handle, 1 if enable else 0), "sem_kernel_timing")

    def kernel_timing_read(self):
        n = C.c_int64()
        ms = C.c_double()
        check(sem_kernel_timing_read(self.handle, C.byref(n), C.byref(ms)), "sem_kernel_timing_read")
        return n.value, ms.value

    def laplace_solve(self, eta, etax, phis, phi, opts=None, stream=None):
        st = sem_solve_stats()
        o = opts if opts is not None else default_opts()
        code = sem_laplace_solve(self.handle, _ptr(eta), _ptr(etax), _ptr(phis), _ptr(phi), C.byref(o),
                                 C.byref(st), _stream(stream))
        check(code, "sem_laplace_solve")
        return st.as_dict()

    def gradient_recover(self, kind, inp, eta, out, stream=None):
        check(sem_gradient_recover(self.handle, kind, _ptr(inp), _ptr(eta) if eta is not None else None,
                                   _ptr(out), _stream(stream)), "sem_gradient_recover")

    def recover_kinematics(self, Phi, eta, etax, u, w, stream=None):
        """u and w at every node (either may be None)."""
        check(sem_recover_kinematics(self.handle, _ptr(Phi), _ptr(eta), _ptr(etax),
                                     _ptr(u) if u is not None else None, _ptr(w) if w is not None else None,
                                     _stream(stream)), "sem_recover_kinematics")

    def free_surface_rhs(self, eta, etax, phix, ws, deta, dphi, stream=None):
        check(sem_free_surface_rhs(self.handle, _ptr(eta), _ptr(etax), _ptr(phix), _ptr(ws), _ptr(deta),
                                   _ptr(dphi), _stream(stream)), "sem_free_surface_rhs")

    def free_surface_rhs_noalloc(self, eta, etax, phix, ws, deta, dphi, stream=None):
        """sem_free_surface_rhs with its scratch in the library's static
        device array (no allocation, no synchronisation)."""
        check(sem_free_surface_rhs_noalloc(self.handle, _ptr(eta), _ptr(etax), _ptr(phix), _ptr(ws), _ptr(deta),
                                           _ptr(dphi), _stream(stream)), "sem_free_surface_rhs_noalloc")

    def rk4_step(self, eta, phis, phi_ws, dt, opts=None, stream=None, raise_on_error=True):
        st = (sem_solve_stats * 4)()
        o = opts if opts is not None else default_opts(warm_start=1)
        code = sem_rk4_step(self.handle, _ptr(eta), _ptr(phis), _ptr(phi_ws), float(dt), C.byref(o), st,
                            _stream(stream))
        if raise_on_error:
            check(code, "sem_rk4_step")
        return code, [s.as_dict() for s in st]

    def set_relaxation(self, weight):
        """Relaxation-zone weights 1 - gamma at the surface nodes (None: off)."""
        if weight is None:
            check(sem_set_relaxation(self.handle, None), "sem_set_relaxation")
            return
        self._relax = np.ascontiguousarray(weight, dtype=np.float64)
        check(sem_set_relaxation(self.handle, self._relax.ctypes.data_as(_D)), "sem_set_relaxation")

    def rk4_step_forced(self, eta, phis, phi_ws, dt, qa, opts=None, stream=None, raise_on_error=True):
        """RK4 step with the relaxation source; qa: device tensor [3, 2, ns]."""
        st = (sem_solve_stats * 4)()
        o = opts if opts is not None else default_opts(warm_start=1)
        code = sem_rk4_step_forced(self.handle, _ptr(eta), _ptr(phis), _ptr(phi_ws), float(dt), _ptr(qa),
                                   C.byref(o), st, _stream(stream))
        if raise_on_error:
            check(code, "sem_rk4_step_forced")
        return code, [s.as_dict() for s in st]

    def reset_history(self, stream=None):
        """Forget the recorded stage solutions (a new initial condition follows)."""
        check(sem_rk4_reset_history(self.handle, _stream(stream)), "sem_rk4_reset_history")

    def __del__(self):
        h = getattr(self, "handle", None)
        if h is not None and h.value and sem_mesh_destroy is not None:
            sem_mesh_destroy(h)
            self.handle = None


class Batch:
    """sem_batch_*: advance several bound meshes per call.

    nstreams = 0: lockstep (one batched GMRES over all tanks); nstreams >= 1:
    each tank's own step on that many concurrent streams."""

    def __init__(self, meshes, nstreams=0, stream=None):
        self.meshes = list(meshes)
        self.nstreams = int(nstreams)
        arr = (C.c_void_p * len(self.meshes))(*[m.handle.value for m in self.meshes])
        self.handle = C.c_void_p()
        check(sem_batch_create(arr, len(self.meshes), self.nstreams, _stream(stream), C.byref(self.handle)),
              "sem_batch_create")

    def graphs(self, enable):
        """Lockstep Arnoldi steps as HIP graph launches (default) or direct launches."""
        check(sem_batch_graphs(self.handle, 1 if enable else 0), "sem_batch_graphs")

    def apply_timed(self, order, prec=SEM_PREC_FP64, reps=20, stream=None):
        """Mean ms of one batched stiffness launch over the tanks of `order`."""
        ms = C.c_float()
        check(sem_batch_apply_timed(self.handle, int(order), int(prec), int(reps), C.byref(ms), _stream(stream)),
              "sem_batch_apply_timed")
        return ms.value

    def graph_count(self):
        c = C.c_int32()
        check(sem_batch_graph_count(self.handle, C.byref(c)), "sem_batch_graph_count")
        return c.value

    def _ptrs(self, tensors):
        return (C.c_void_p * len(self.meshes))(*[t.data_ptr() for t in tensors])

    def _active(self, active):
        n = len(self.meshes)
        return None if active is None else (C.c_uint8 * n)(*[1 if a else 0 for a in active])

    def rk4_step(self, etas, phis, phiws, dts, active=None, opts=None, stream=None):
        n = len(self.meshes)
        dt = (C.c_double * n)(*[float(v) for v in dts])
        st = (C.c_int32 * n)()
        it = (C.c_int32 * n)()
        o = opts if opts is not None else default_opts(warm_start=1)
        code = sem_batch_rk4_step(self.handle, self._ptrs(etas), self._ptrs(phis), self._ptrs(phiws), dt,
                                  self._active(active), C.byref(o), st, it, _stream(stream))
        return code, list(st), list(it)

    def laplace_solve(self, etas, etaxs, phiss, phis_out, active=None, opts=None, stream=None):
        n = len(self.meshes)
        st = (C.c_int32 * n)()
        it = (C.c_int32 * n)()
        o = opts if opts is not None else default_opts()
        code = sem_batch_laplace_solve(self.handle, self._ptrs(etas), self._ptrs(etaxs), self._ptrs(phiss),
                                       self._ptrs(phis_out), self._active(active), C.byref(o), st, it,
                                       _stream(stream))
        return code, list(st), list(it)

    def __del__(self):
        h = getattr(self, "handle", None)
        if h is not None and h.value and sem_batch_destroy is not None:
            sem_batch_destroy(h)
            self.handle = None


def reference_operators(P, Pf, ic=2, sigma_f=1.0):
    """The host's reference-element operators (sem_reference_operators)."""
    Np = (P + 1) * (P + 2) // 2
    out = dict(r=np.empty(Np), s=np.empty(Np), Dr=np.empty((Np, Np)), Ds=np.empty((Np, Np)), M=np.empty((Np, Np)),
               F=np.empty((P + 1, P + 1)), I=np.empty((Pf + 1, P + 1)), Mf=np.empty((Pf + 1, Pf + 1)))
    args = [out[k].ctypes.data_as(_D) for k in ("r", "s", "Dr", "Ds", "M", "F", "I", "Mf")]
    check(sem_reference_operators(P, Pf, ic, float(sigma_f), *args), "sem_reference_operators")
    return out


def mesh_from_spec(spec, h, hx, **kw):
    return Mesh(spec.nx, spec.nz, spec.P, spec.length, spec.periodic, h, hx, g=spec.g,
                filter_ic=spec.filter_ic, filter_sigma=spec.filter_sigma, overint=spec.Pf, **kw)
