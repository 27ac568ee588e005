"""ctypes binding of include/ldg.h with the same entry-point names.

Argument marshalling only: numpy arrays for host inputs, torch tensors on the
GPU for device buffers (``data_ptr()``), the current torch stream as the HIP
stream.  Every step of the method runs inside libldg.so.
"""
import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))

LDG_FP64, LDG_MIXED_FP32, LDG_MIXED_BF16 = 0, 1, 2
LDG_PC_BLOCK_JACOBI, LDG_PC_GNN = 0, 1
STATUS = {0: "OK", -1: "EINVAL", -2: "EMESH", -3: "ENOMEM", -4: "EDEVICE", -5: "ENOCONV",
          -6: "EUNSUPPORTED", -7: "EIO", -8: "ECALLBACK"}


class LdgError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("%s: %s" % (STATUS.get(code, code), msg))
        self.code = code


class Options(C.Structure):
    _fields_ = [("p", C.c_int), ("eta", C.c_double), ("precision", C.c_int),
                ("precond", C.c_int), ("rtol", C.c_double), ("restart", C.c_int),
                ("max_iters", C.c_int), ("stream", C.c_void_p), ("krylov", C.c_int),
                ("inner_rtol", C.c_double), ("quad", C.c_int),
                ("cg_keep_direction", C.c_int), ("edge_traces", C.c_int)]


class Sizes(C.Structure):
    _fields_ = [("K", C.c_int64), ("N", C.c_int), ("R", C.c_int), ("R1", C.c_int),
                ("n_bnd", C.c_int64), ("E_int", C.c_int64)]


class KernelStat(C.Structure):
    _fields_ = [("launches", C.c_int64), ("total_ms", C.c_double), ("bytes", C.c_double),
                ("flops", C.c_double)]


KERNELS = ["div", "grad", "bj_apply", "assemble", "bj_setup", "krylov", "project", "gnn", "factor",
           "mf", "residual"]


class StepInfo(C.Structure):
    _fields_ = [("iters", C.c_int), ("restarts", C.c_int), ("ir_steps", C.c_int),
                ("fallbacks", C.c_int), ("krylov", C.c_int), ("rel_residual", C.c_double),
                ("t", C.c_double), ("learned_iters", C.c_int), ("guarded_iters", C.c_int),
                ("fallback_reason", C.c_int), ("bdf_order", C.c_int),
                ("gmres_restart", C.c_int)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


_P = C.c_void_p
_DP = C.POINTER(C.c_double)
FIELD_FN = C.CFUNCTYPE(C.c_int, _P, C.c_double, _DP, _DP, _DP, C.c_int64)
FLUX_FN = C.CFUNCTYPE(C.c_int, _P, C.c_double, _DP, _DP, _DP, _DP, _DP, C.c_int64)


class Problem(C.Structure):
    _fields_ = [("d", FIELD_FN), ("f", FIELD_FN), ("c_D", FIELD_FN), ("g_N", FLUX_FN),
                ("user", _P)]


def _field(fn):
    """C callback from fn(t, x, y) -> values (numpy); an exception returns 1."""
    if fn is None:
        return FIELD_FN()

    def cb(user, t, x, y, out, n):
        try:
            xs, ys = np.ctypeslib.as_array(x, (n,)), np.ctypeslib.as_array(y, (n,))
            np.ctypeslib.as_array(out, (n,))[:] = fn(t, xs, ys)
            return 0
        except Exception:
            return 1
    return FIELD_FN(cb)


def _flux(fn):
    """C callback from fn(t, x, y, nx, ny) -> values (numpy); an exception returns 1."""
    if fn is None:
        return FLUX_FN()

    def cb(user, t, x, y, nx, ny, out, n):
        try:
            a = [np.ctypeslib.as_array(v, (n,)) for v in (x, y, nx, ny)]
            np.ctypeslib.as_array(out, (n,))[:] = fn(t, *a)
            return 0
        except Exception:
            return 1
    return FLUX_FN(cb)


_SIGS = {
    "ldg_options_default": [C.POINTER(Options)],
    "ldg_create": [_P, C.c_int64, _P, C.c_int64, _P, C.POINTER(Options), C.POINTER(_P)],
    "ldg_get_sizes": [_P, C.POINTER(Sizes)],
    "ldg_quad_points": [_P, C.c_int, _P, _P],
    "ldg_project": [_P, _P, _P],
    "ldg_set_state": [_P, _P, C.c_int, C.c_double],
    "ldg_set_initial_samples": [_P, _P, C.c_double],
    "ldg_step_sampled": [_P, C.c_double, _P, _P, _P, _P, C.POINTER(StepInfo)],
    "ldg_solve_stationary_sampled": [_P, _P, _P, _P, _P, C.POINTER(StepInfo)],
    "ldg_get_solution": [_P, _P, _P, _P, C.c_int],
    "ldg_assemble": [_P, _P],
    "ldg_get_blocks": [_P, _P],
    "ldg_get_blocks_lowp": [_P, _P],
    "ldg_get_blocks_rows": [_P, _P, C.c_int64, _P],
    "ldg_get_bj_rows": [_P, _P, C.c_int64, _P],
    "ldg_apply_schur": [_P, C.c_double, _P, _P],
    "ldg_apply_schur_lowp": [_P, C.c_double, _P, _P],
    "ldg_apply_schur_noalloc": [_P, C.c_double, _P, _P],
    "ldg_apply_full": [_P, C.c_double, _P, _P],
    "ldg_bj_setup": [_P, C.c_double],
    "ldg_get_bj": [_P, _P],
    "ldg_gnn_num_params": [_P, C.POINTER(C.c_int64)],
    "ldg_gnn_set_params": [_P, _P, C.c_int64],
    "ldg_gnn_get_params": [_P, _P, C.c_int64],
    "ldg_gnn_set_context": [_P, _P, C.c_double],
    "ldg_gnn_forward": [_P, _P, _P],
    "ldg_gnn_set_mode": [_P, C.c_int],
    "ldg_gnn_factor_omega": [_P, _P],
    "ldg_gnn_factor_export": [_P, _P, _P],
    "ldg_gnn_factor_storage": [_P, C.c_int],
    "ldg_gnn_factor_export_rows": [_P, _P, C.c_int64, _P, _P],
    "ldg_set_time_scheme": [_P, C.c_int],
    "ldg_set_history": [_P, _P, C.c_double],
    "ldg_gnn_set_loss": [_P, C.c_int],
    "ldg_gnn_loss_grad": [_P, _P, _P, _P, C.POINTER(C.c_double)],
    "ldg_gnn_train_step": [_P, _P, _P, C.c_double, C.POINTER(C.c_double)],
    "ldg_gnn_collect": [_P, C.c_int, _P, _P, _P],
    "ldg_gnn_collected": [_P, C.POINTER(C.c_int)],
    "ldg_set_timing": [_P, C.c_int],
    "ldg_set_matrix_free": [_P, C.c_int],
    "ldg_get_kernel_stat": [_P, C.c_int, C.POINTER(KernelStat)],
    "ldg_sample_workload": [_P, C.c_int, C.c_double, _P, _P, _P, _P, _P, _P],
    "ldg_lagrange": [_P, _P, _P, C.POINTER(C.c_int)],
    "ldg_set_initial": [_P, FIELD_FN, _P],
    "ldg_step": [_P, C.c_double, C.POINTER(Problem), C.POINTER(StepInfo)],
    "ldg_set_initial_dofs": [_P, _P, C.c_int],
    "ldg_gnn_load": [_P, _P, C.c_int64],
    "ldg_gnn_save": [_P, _P, C.c_int64],
    "ldg_write_vtu": [_P, C.c_char_p, C.c_char_p, _P, C.c_int, C.c_int],
    "ldg_mesh_read_medit": [C.c_char_p, C.POINTER(C.c_int64), C.POINTER(C.c_int64), _P, _P, _P],
    "ldg_edge_kinds_from_ids": [C.c_int64, _P, _P, C.c_int, _P],
}

_lib = None


def library_path():
    return os.path.join(HERE, "libldg.so")


def load_library():
    """Load libldg.so from this package directory; raise if it is not built."""
    global _lib
    if _lib is not None:
        return _lib
    path = library_path()
    if not os.path.exists(path):
        raise RuntimeError("libldg.so is not built; run `python -m paper_1408_3877_amd.build`")
    # torch first: the library then binds to the HIP runtime torch has loaded, so
    # that the process holds one runtime (loaded the other way round, torch's
    # runtime reports no device)
    import torch  # noqa: F401
    lib = C.CDLL(path)
    for name, args in _SIGS.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = C.c_int
    lib.ldg_destroy.argtypes = [_P]
    lib.ldg_destroy.restype = None
    lib.ldg_last_error.argtypes = [_P]
    lib.ldg_last_error.restype = C.c_char_p
    _lib = lib
    return lib


def _ptr(t):
    return None if t is None else C.c_void_p(t.data_ptr())


def _check_noctx(lib, code):
    if code != 0:
        raise LdgError(code, lib.ldg_last_error(None).decode())


def read_mesh_medit(path):
    """(coordV numV x 2, V0T K x 3 0-based counter-clockwise, edge_id K x 3) of
    a MEDIT .mesh file; edge_id is 0 on interior edges, the boundary ID on
    boundary edges, -1 where the file lists none."""
    lib = load_library()
    nv, nk = C.c_int64(0), C.c_int64(0)
    p = os.fsencode(path)
    _check_noctx(lib, lib.ldg_mesh_read_medit(p, C.byref(nv), C.byref(nk), None, None, None))
    coordV = np.zeros((nv.value, 2), np.float64)
    V0T = np.zeros((nk.value, 3), np.int32)
    ids = np.zeros((nk.value, 3), np.int32)
    _check_noctx(lib, lib.ldg_mesh_read_medit(p, C.byref(nv), C.byref(nk), coordV.ctypes.data,
                                              V0T.ctypes.data, ids.ctypes.data))
    return coordV, V0T, ids


def edge_kinds_from_ids(edge_id, neumann_ids=()):
    """ldg_edge_kind per local edge: 0 interior, Neumann for the listed IDs,
    Dirichlet otherwise."""
    lib = load_library()
    ids = np.ascontiguousarray(edge_id, np.int32)
    neu = np.ascontiguousarray(list(neumann_ids) or [0], np.int32)
    kind = np.zeros(ids.shape, np.int8)
    _check_noctx(lib, lib.ldg_edge_kinds_from_ids(ids.shape[0], ids.ctypes.data, neu.ctypes.data,
                                                  len(neumann_ids), kind.ctypes.data))
    return kind


class Solver:
    """One LDG context: a mesh, an order p and the solver options."""

    def __init__(self, coordV, V0T, edge_kind, p, eta=1.0, precision=LDG_FP64,
                 precond=LDG_PC_BLOCK_JACOBI, rtol=1e-8, restart=30, max_iters=5000,
                 krylov=0, inner_rtol=1e-3, device=None, quad="exact", keep_direction=True,
                 edge_traces=True):
        import torch
        self.torch = torch
        self.lib = load_library()
        if not torch.cuda.is_available():
            raise RuntimeError("no GPU visible: the LDG library runs on the device only")
        self.device = torch.device("cuda", torch.cuda.current_device() if device is None else device)
        coordV = np.ascontiguousarray(coordV, dtype=np.float64)
        V0T = np.ascontiguousarray(V0T, dtype=np.int32)
        kind = np.ascontiguousarray(edge_kind, dtype=np.int8)
        opt = Options()
        self.lib.ldg_options_default(C.byref(opt))
        opt.p, opt.eta, opt.precision, opt.precond = p, eta, precision, precond
        opt.rtol, opt.restart, opt.max_iters, opt.krylov = rtol, restart, max_iters, krylov
        opt.inner_rtol = inner_rtol
        opt.quad = {"exact": 0, "paper": 1}.get(quad, quad)
        opt.cg_keep_direction = int(bool(keep_direction))
        opt.edge_traces = int(bool(edge_traces))
        with torch.cuda.device(self.device):
            opt.stream = C.c_void_p(torch.cuda.current_stream().cuda_stream)
            h = C.c_void_p()
            code = self.lib.ldg_create(coordV.ctypes.data, coordV.shape[0], V0T.ctypes.data,
                                       V0T.shape[0], kind.ctypes.data, C.byref(opt), C.byref(h))
        self.h = h
        if code != 0:
            msg = self.lib.ldg_last_error(h).decode() if h.value else ""
            if h.value:
                self.lib.ldg_destroy(h)
            self.h = None
            raise LdgError(code, msg)
        s = Sizes()
        self._check(self.lib.ldg_get_sizes(self.h, C.byref(s)))
        self.K, self.N, self.R, self.R1 = s.K, s.N, s.R, s.R1
        self.n_bnd, self.E_int = s.n_bnd, s.E_int
        self.p = p

    # -- helpers ---------------------------------------------------------------
    def _check(self, code):
        if code != 0:
            raise LdgError(code, self.lib.ldg_last_error(self.h).decode())

    def _dev(self, x, shape=None):
        t = self.torch
        if not isinstance(x, t.Tensor):
            x = t.as_tensor(np.asarray(x, dtype=np.float64))
        if shape is not None and tuple(x.shape) != tuple(shape):
            raise ValueError("expected shape %s, got %s" % (tuple(shape), tuple(x.shape)))
        if x.dtype not in (t.float64, t.float32):
            raise TypeError("expected a floating-point array, got %s" % x.dtype)
        return x.to(device=self.device, dtype=t.float64).contiguous()

    def _sampled_inputs(self, d, f, cD, gN):
        """Check and place the sampled data of a step: d, f at the R*K volume
        points, c_D and g_N (optional) at the R1*n_bnd boundary-edge points."""
        nv, nb = (self.R * self.K,), (self.R1 * self.n_bnd,)
        return (self._dev(d, nv), self._dev(f, nv),
                None if cD is None else self._dev(cD, nb),
                None if gN is None else self._dev(gN, nb))

    def _empty(self, *shape):
        return self.torch.empty(*shape, dtype=self.torch.float64, device=self.device)

    def close(self):
        if getattr(self, "h", None):
            self.lib.ldg_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- entry points ---------------------------------------------------------
    def quad_points(self, kind):
        n = self.R * self.K if kind == 0 else self.R1 * self.n_bnd
        x, y = self._empty(max(n, 1)), self._empty(max(n, 1))
        self._check(self.lib.ldg_quad_points(self.h, kind, _ptr(x), _ptr(y)))
        return x[:n], y[:n]

    def project(self, samples):
        s = self._dev(samples, (self.R * self.K,))
        out = self._empty(self.K, self.N)
        self._check(self.lib.ldg_project(self.h, _ptr(s), _ptr(out)))
        return out

    def set_state(self, Cm, t):
        Cd = self._dev(Cm, (self.K, self.N))
        self._check(self.lib.ldg_set_state(self.h, _ptr(Cd), 1, float(t)))

    def set_initial_samples(self, c0, t0=0.0):
        s = self._dev(c0, (self.R * self.K,))
        self._check(self.lib.ldg_set_initial_samples(self.h, _ptr(s), float(t0)))

    def step_sampled(self, dt, d, f, cD=None, gN=None):
        d, f, cD, gN = self._sampled_inputs(d, f, cD, gN)
        info = StepInfo()
        code = self.lib.ldg_step_sampled(self.h, float(dt), _ptr(d), _ptr(f), _ptr(cD), _ptr(gN),
                                         C.byref(info))
        if code != 0:
            # the library fills info on LDG_ENOCONV too (state not advanced)
            err = LdgError(code, self.lib.ldg_last_error(self.h).decode())
            err.info = info.as_dict()
            raise err
        return info.as_dict()

    def set_matrix_free(self, on=True):
        """Apply the operator without streaming stored blocks (matrix cores)."""
        self._check(self.lib.ldg_set_matrix_free(self.h, int(bool(on))))

    def lagrange(self, Cm=None):
        """Values at the Lagrange points (K x nL) of Cm (K x N), or of the state."""
        nl = C.c_int(0)
        self._check(self.lib.ldg_lagrange(self.h, None, None, C.byref(nl)))
        Cd = None if Cm is None else self._dev(Cm, (self.K, self.N))
        out = self._empty(self.K, nl.value)
        self._check(self.lib.ldg_lagrange(self.h, _ptr(Cd), _ptr(out), C.byref(nl)))
        return out

    def write_vtu(self, path, name, lagr, binary=False):
        """Write Lagrange values (K x nL) as a .vtu file."""
        v = np.ascontiguousarray(lagr.detach().cpu().numpy() if hasattr(lagr, "detach") else lagr,
                                 np.float64)
        self._check(self.lib.ldg_write_vtu(self.h, os.fsencode(path), name.encode(), v.ctypes.data,
                                           v.shape[1], int(bool(binary))))

    def set_initial(self, c0):
        """Initial state from a host function c0(t, x, y) (called with t = 0)."""
        cb = _field(c0)
        self._check(self.lib.ldg_set_initial(self.h, cb, None))

    def step(self, dt, d, f, c_D=None, g_N=None):
        """One step with host field functions d, f, c_D (t, x, y) and g_N
        (t, x, y, nx, ny) evaluated by the library at its own points at t + dt."""
        cbs = (_field(d), _field(f), _field(c_D), _flux(g_N))
        pb = Problem(cbs[0], cbs[1], cbs[2], cbs[3], None)
        info = StepInfo()
        code = self.lib.ldg_step(self.h, float(dt), C.byref(pb), C.byref(info))
        self._check(code)
        return info.as_dict()

    def solve_stationary_sampled(self, d, f, cD=None, gN=None):
        """A Y = V from sampled data (no mass term, no history); the solution
        becomes the state."""
        d, f, cD, gN = self._sampled_inputs(d, f, cD, gN)
        info = StepInfo()
        code = self.lib.ldg_solve_stationary_sampled(self.h, _ptr(d), _ptr(f), _ptr(cD), _ptr(gN),
                                                     C.byref(info))
        self._check(code)
        return info.as_dict()

    def set_time_scheme(self, scheme):
        """"euler" (0) or "bdf2" (1)."""
        k = {"euler": 0, "bdf2": 1}.get(scheme, scheme)
        self._check(self.lib.ldg_set_time_scheme(self.h, int(k)))

    def set_history(self, C_prev, dt_prev):
        Cd = self._dev(C_prev, (self.K, self.N))
        self._check(self.lib.ldg_set_history(self.h, _ptr(Cd), float(dt_prev)))

    def get_solution(self):
        Cm, Z1, Z2 = self._empty(self.K, self.N), self._empty(self.K, self.N), self._empty(self.K, self.N)
        self._check(self.lib.ldg_get_solution(self.h, _ptr(Cm), _ptr(Z1), _ptr(Z2), 1))
        return Cm, Z1, Z2

    def assemble(self, D):
        Dd = self._dev(D, (self.K, self.N))
        self._check(self.lib.ldg_assemble(self.h, _ptr(Dd)))

    def get_blocks(self):
        out = self._empty(self.K, 5, self.N, self.N)
        self._check(self.lib.ldg_get_blocks(self.h, _ptr(out)))
        return out

    def _rows(self, fn, elems, ns):
        e = np.ascontiguousarray(elems, dtype=np.int32)
        if e.size and (e.min() < 0 or e.max() >= self.K):
            raise ValueError("element index out of range")
        ed = self.torch.as_tensor(e).to(self.device)
        out = self._empty(max(len(e), 1), ns, self.N, self.N)[:len(e)]
        self._check(fn(self.h, _ptr(ed), len(e), _ptr(out)))
        return out

    def get_blocks_rows(self, elems):
        return self._rows(self.lib.ldg_get_blocks_rows, elems, 5)

    def get_bj_rows(self, elems):
        return self._rows(self.lib.ldg_get_bj_rows, elems, 1)[:, 0]

    def get_blocks_lowp(self):
        out = self._empty(self.K, 5, self.N, self.N)
        self._check(self.lib.ldg_get_blocks_lowp(self.h, _ptr(out)))
        return out

    def apply_schur(self, dt, Cm):
        Cd = self._dev(Cm, (self.K, self.N))
        y = self._empty(self.K, self.N)
        self._check(self.lib.ldg_apply_schur(self.h, float(dt), _ptr(Cd), _ptr(y)))
        return y

    def apply_schur_lowp(self, dt, Cm):
        """The eliminated operator in the inner precision (FP32 vectors, FP32 or
        BF16 blocks) of a mixed-precision context, widened to FP64."""
        Cd = self._dev(Cm, (self.K, self.N))
        y = self._empty(self.K, self.N)
        self._check(self.lib.ldg_apply_schur_lowp(self.h, float(dt), _ptr(Cd), _ptr(y)))
        return y

    def apply_schur_noalloc(self, dt, Cm, y):
        """apply_schur into the caller's y (device K x N FP64) through the
        allocation-free entry point (library workspace, no allocation)."""
        Cd = self._dev(Cm, (self.K, self.N))
        t = self.torch
        if (not isinstance(y, t.Tensor) or tuple(y.shape) != (self.K, self.N) or
                y.dtype != t.float64 or y.device != self.device or not y.is_contiguous()):
            raise ValueError("y must be a contiguous float64 device tensor of shape (K, N)")
        self._check(self.lib.ldg_apply_schur_noalloc(self.h, float(dt), _ptr(Cd), _ptr(y)))
        return y

    def apply_full(self, dt, Y):
        Yd = self._dev(Y, (3 * self.K * self.N,))
        out = self._empty(3 * self.K * self.N)
        self._check(self.lib.ldg_apply_full(self.h, float(dt), _ptr(Yd), _ptr(out)))
        return out

    def bj_setup(self, dt):
        self._check(self.lib.ldg_bj_setup(self.h, float(dt)))

    def get_bj(self):
        out = self._empty(self.K, self.N, self.N)
        self._check(self.lib.ldg_get_bj(self.h, _ptr(out)))
        return out

    # -- learned preconditioner ------------------------------------------------
    def gnn_num_params(self):
        n = C.c_int64()
        self._check(self.lib.ldg_gnn_num_params(self.h, C.byref(n)))
        return n.value

    def gnn_set_params(self, w):
        w = np.ascontiguousarray(w, dtype=np.float32)
        self._check(self.lib.ldg_gnn_set_params(self.h, w.ctypes.data, w.size))

    def gnn_get_params(self):
        w = np.zeros(self.gnn_num_params(), dtype=np.float32)
        self._check(self.lib.ldg_gnn_get_params(self.h, w.ctypes.data, w.size))
        return w

    def gnn_set_mode(self, mode):
        """0 / "correction": per-iteration residual correction (flexible CG);
        1 / "factor": linear factored preconditioner built once per system."""
        m = {"correction": 0, "factor": 1}.get(mode, mode)
        self._check(self.lib.ldg_gnn_set_mode(self.h, int(m)))

    def gnn_factor_storage(self, kind):
        """"f32", "bf16", "fp8" (default: W in BF16, O in FP8) or "fp8w" (both in FP8, W with a
        power-of-two scale per triangle) storage of the factor blocks."""
        self._check(self.lib.ldg_gnn_factor_storage(
            self.h, {"f32": 0, "bf16": 1, "fp8": 2, "fp8w": 3}[kind]))

    def gnn_factor_omega(self):
        om = self.torch.empty((self.K, 3), dtype=self.torch.float32, device=self.device)
        self._check(self.lib.ldg_gnn_factor_omega(self.h, _ptr(om)))
        return om

    def gnn_factor_export(self):
        t = self.torch
        blk = t.empty((self.K, 4, self.N, self.N), dtype=t.float64, device=self.device)
        ln = t.empty((self.K, 3), dtype=t.float32, device=self.device)
        self._check(self.lib.ldg_gnn_factor_export(self.h, _ptr(blk), _ptr(ln)))
        return blk, ln

    def gnn_factor_export_rows(self, elems):
        t = self.torch
        el = t.as_tensor(np.asarray(elems, dtype=np.int32), device=self.device)
        blk = t.empty((len(el), 4, self.N, self.N), dtype=t.float64, device=self.device)
        ln = t.empty((len(el), 3), dtype=t.float32, device=self.device)
        self._check(self.lib.ldg_gnn_factor_export_rows(self.h, _ptr(el), len(el), _ptr(blk), _ptr(ln)))
        return blk, ln

    def gnn_set_loss(self, kind):
        """0 / "mse": mean squared error; 1 / "energy": energy norm relative to the
        block-Jacobi step's; 2 / "frobenius": probe estimate of ||G S G^T - I||_F^2
        (factored mode; the probe is passed as rhat); 3 / "optstep": energy left
        after one preconditioned step with the best step length (factored mode)."""
        k = {"mse": 0, "energy": 1, "frobenius": 2, "optstep": 3}.get(kind, kind)
        self._check(self.lib.ldg_gnn_set_loss(self.h, int(k)))

    def gnn_set_context(self, D, dt):
        Dd = None if D is None else self._dev(D, (self.K, self.N))
        self._check(self.lib.ldg_gnn_set_context(self.h, _ptr(Dd), float(dt)))

    def _f32(self, x):
        t = self.torch
        if not isinstance(x, t.Tensor):
            x = t.as_tensor(np.asarray(x, dtype=np.float32))
        return x.to(device=self.device, dtype=t.float32).contiguous()

    def gnn_forward(self, rhat):
        r = self._f32(rhat)
        out = self.torch.empty_like(r)
        self._check(self.lib.ldg_gnn_forward(self.h, _ptr(r), _ptr(out)))
        return out

    def gnn_loss_grad(self, rhat, target):
        r, t = self._f32(rhat), self._f32(target)
        g = self.torch.empty(self.gnn_num_params(), dtype=self.torch.float32, device=self.device)
        loss = C.c_double()
        self._check(self.lib.ldg_gnn_loss_grad(self.h, _ptr(r), _ptr(t), _ptr(g), C.byref(loss)))
        return loss.value, g

    def gnn_train_step(self, rhat, target, lr):
        r, t = self._f32(rhat), self._f32(target)   # keep both alive across the call
        loss = C.c_double()
        self._check(self.lib.ldg_gnn_train_step(self.h, _ptr(r), _ptr(t), float(lr), C.byref(loss)))
        return loss.value

    def gnn_collect(self, iters):
        it = np.ascontiguousarray(iters, dtype=np.int32)
        shape = (len(it), self.K, self.N)
        r = self.torch.empty(shape, dtype=self.torch.float32, device=self.device)
        t = self.torch.empty(shape, dtype=self.torch.float32, device=self.device)
        self._check(self.lib.ldg_gnn_collect(self.h, len(it), it.ctypes.data, _ptr(r), _ptr(t)))
        self._collect_bufs = (r, t)
        return r, t

    def gnn_collected(self):
        n = C.c_int()
        self._check(self.lib.ldg_gnn_collected(self.h, C.byref(n)))
        return n.value

    def set_timing(self, on):
        self._check(self.lib.ldg_set_timing(self.h, int(bool(on))))

    def kernel_stats(self):
        out = {}
        for i, name in enumerate(KERNELS):
            st = KernelStat()
            self._check(self.lib.ldg_get_kernel_stat(self.h, i, C.byref(st)))
            out[name] = {"launches": st.launches, "total_ms": st.total_ms, "bytes": st.bytes,
                         "flops": st.flops}
        return out

    def sample_workload(self, kind, t, dT=None, want=("d", "f", "cD", "gN")):
        dTd = None if dT is None else self._dev(dT, (self.K,))
        nv, nbd = self.R * self.K, self.R1 * self.n_bnd
        out = {}
        for name, n in (("d", nv), ("f", nv), ("cD", nbd), ("gN", nbd), ("c0", nv)):
            out[name] = self._empty(max(n, 1))[:n] if name in want else None
        self._check(self.lib.ldg_sample_workload(
            self.h, int(kind), float(t), _ptr(dTd), _ptr(out["d"]), _ptr(out["f"]),
            _ptr(out["cD"]), _ptr(out["gN"]), _ptr(out["c0"])))
        return out
