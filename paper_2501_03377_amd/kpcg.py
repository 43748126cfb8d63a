"""ctypes binding of the kpcg C ABI (include/kpcg.h).

Argument marshalling only: every step of a solve runs in the HIP library.
The raw entry points keep the C names (kp_plan_create, kp_solve, ...); the
`Plan` class wraps them for torch tensors.  PyTorch is used only for device
memory and streams.  If the library has not been built this module raises
on import: there is no fallback path.
"""

import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libkpcg.so")

BC = {"P": 0, "D": 1, "N": 2, "DN": 3, "ND": 4}
PREC = {"f64": 0, "f32": 1, "bf16": 2, "bf16x6": 3, "i8x7": 4, "i8x6": 5}

KP_OK = 0
KP_NOT_CONVERGED = 1
KP_EINVAL = -1
KP_ENOMEM = -2
KP_EHIP = -3
KP_ENONFINITE = -4
KP_EBREAKDOWN = -5
KP_EBUSY = -6

KP_FLAG_NO_PRECOND = 1
KP_FLAG_FLEX_BETA = 2
KP_FLAG_RESIDUAL_ONLY = 4
KP_FLAG_NO_GRAPH = 8
KP_FLAG_DIAGNOSTICS = 16
KP_FLAG_ANORM_STOP = 32
KP_FLAG_WARM_START = 64
KP_DIAG_COLUMNS = 7
# Columns of kp_plan_diagnostics.
DIAG_COLUMNS = ("true_rel_res", "rel_res", "kappa", "error_proxy", "null_component",
                "hs_term", "hs_error_estimate")

# Every symbol declared in include/kpcg.h.
EXPORTS = (
    "kp_basis_1d", "kp_plan_create", "kp_plan_destroy", "kp_plan_workspace_bytes",
    "kp_plan_resident_bytes", "kp_plan_set_workspace", "kp_plan_set_stream",
    "kp_apply_laplacian", "kp_apply_pinv", "kp_solve", "kp_strerror", "kp_version",
    "kp_plan_set_profiling", "kp_plan_profile", "kp_plan_profile_reset", "kp_kernel_class_name",
    "kp_plan_autotune", "kp_plan_time_kernel", "kp_plan_get_tuning", "kp_plan_set_tuning", "kp_plan_graph_count",
    "kp_tile_shape", "kp_server_create", "kp_server_submit", "kp_server_poll", "kp_server_now",
    "kp_server_stats_get", "kp_server_destroy", "kp_server_last_error", "kp_last_error",
    "kp_assemble_rhs", "kp_field", "kp_plan_set_preconditioner", "kp_apply_preconditioner",
    "kp_plan_diagnostics", "kp_lowrank_table", "kp_solve_async", "kp_poll", "kp_wait",
    "kp_apply_pinv_noalloc",
)
KP_NOALLOC_SCRATCH_BYTES = 64 << 20
KERNEL_CLASSES = 18


class KpResult(ctypes.Structure):
    _fields_ = [
        ("status", ctypes.c_int32),
        ("iterations", ctypes.c_int32),
        ("pinv_applications", ctypes.c_int32),
        ("reserved", ctypes.c_int32),
        ("rel_res", ctypes.c_double),
        ("true_rel_res", ctypes.c_double),
        ("err_est", ctypes.c_double),
        ("removed_mean", ctypes.c_double),
    ]

    def as_dict(self):
        return {name: getattr(self, name) for name, _ in self._fields_ if name != "reserved"}


class KpError(RuntimeError):
    def __init__(self, status, where):
        self.status = status
        detail = kp_last_error() if status in (-2, -3) else ""
        super().__init__(f"{where}: {kp_strerror(status)} ({status})"
                         + (f" [{detail}]" if detail else ""))


class KpRequest(ctypes.Structure):
    _fields_ = [
        ("id", ctypes.c_int64),
        ("nx", ctypes.c_int), ("ny", ctypes.c_int), ("nz", ctypes.c_int),
        ("bc", ctypes.c_int * 3),
        ("prec", ctypes.c_int),
        ("tol", ctypes.c_double),
        ("max_iter", ctypes.c_int),
        ("flags", ctypes.c_int),
        ("mem", ctypes.c_int),
        ("eta", ctypes.c_void_p),
        ("u", ctypes.c_void_p),
    ]


class KpCompletion(ctypes.Structure):
    _fields_ = [
        ("id", ctypes.c_int64),
        ("status", ctypes.c_int32),
        ("iterations", ctypes.c_int32),
        ("batch", ctypes.c_int32),
        ("worker", ctypes.c_int32),
        ("rel_res", ctypes.c_double),
        ("true_rel_res", ctypes.c_double),
        ("err_est", ctypes.c_double),
        ("t_submit", ctypes.c_double),
        ("t_start", ctypes.c_double),
        ("t_end", ctypes.c_double),
    ]

    def as_dict(self):
        return {name: getattr(self, name) for name, _ in self._fields_}


class KpServerStats(ctypes.Structure):
    _fields_ = [
        ("submitted", ctypes.c_int64), ("completed", ctypes.c_int64),
        ("batches", ctypes.c_int64), ("plans_created", ctypes.c_int64),
        ("plans_evicted", ctypes.c_int64), ("rejected", ctypes.c_int64),
        ("plans_cached", ctypes.c_int32), ("queued", ctypes.c_int32),
        ("hbm_used", ctypes.c_size_t), ("hbm_high_water", ctypes.c_size_t),
        ("hbm_budget", ctypes.c_size_t),
    ]

    def as_dict(self):
        return {name: getattr(self, name) for name, _ in self._fields_}


KP_MEM_DEVICE, KP_MEM_HOST = 0, 1


def _load():
    # torch ships its own HIP runtime under the same soname as the system one
    # this library links.  Imported first, its copy satisfies the library's
    # dependency and the process has one runtime; loaded the other way round,
    # torch pulls in a second copy and one of the two finds no device.
    import torch  # noqa: F401
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with `python paper_2501_03377_amd/build.py`")
    lib = ctypes.CDLL(LIB_PATH)
    vp, i, d, sz = ctypes.c_void_p, ctypes.c_int, ctypes.c_double, ctypes.c_size_t
    pd = ctypes.POINTER(ctypes.c_double)
    sig = {
        "kp_basis_1d": (i, [i, i, pd, pd]),
        "kp_plan_create": (i, [ctypes.POINTER(vp), i, i, i, ctypes.POINTER(ctypes.c_int), i, i, vp]),
        "kp_plan_destroy": (None, [vp]),
        "kp_plan_workspace_bytes": (sz, [vp, i]),
        "kp_plan_resident_bytes": (sz, [vp]),
        "kp_plan_set_workspace": (i, [vp, vp, sz]),
        "kp_plan_set_stream": (i, [vp, vp]),
        "kp_apply_laplacian": (i, [vp, vp, vp, i]),
        "kp_apply_pinv": (i, [vp, vp, vp, i]),
        "kp_apply_pinv_noalloc": (i, [vp, vp, vp, i]),
        "kp_solve": (i, [vp, vp, vp, i, d, i, i, ctypes.POINTER(KpResult), pd]),
        "kp_solve_async": (i, [vp, vp, vp, i, d, i, i, ctypes.POINTER(KpResult), pd,
                               ctypes.POINTER(vp)]),
        "kp_poll": (i, [vp]),
        "kp_wait": (i, [vp]),
        "kp_strerror": (ctypes.c_char_p, [i]),
        "kp_version": (ctypes.c_char_p, []),
        "kp_plan_set_profiling": (i, [vp, i]),
        "kp_plan_profile": (i, [vp, i, pd, ctypes.POINTER(ctypes.c_int64)]),
        "kp_plan_profile_reset": (i, [vp]),
        "kp_kernel_class_name": (ctypes.c_char_p, [i]),
        "kp_plan_autotune": (i, [vp, i, i, ctypes.POINTER(ctypes.c_int)]),
        "kp_plan_time_kernel": (i, [vp, i, i, i, i, pd]),
        "kp_plan_diagnostics": (i, [vp, pd, i, i, i]),
        "kp_lowrank_table": (i, [i, i, i, i, i, pd]),
        "kp_plan_get_tuning": (i, [vp, ctypes.POINTER(ctypes.c_int), i]),
        "kp_plan_set_tuning": (i, [vp, ctypes.POINTER(ctypes.c_int), i]),
        "kp_plan_graph_count": (i, [vp]),
        "kp_tile_shape": (i, [i, i, ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_int),
                              ctypes.POINTER(ctypes.c_int)]),
        "kp_server_create": (i, [ctypes.POINTER(vp), sz, i, i]),
        "kp_server_submit": (i, [vp, ctypes.POINTER(KpRequest)]),
        "kp_server_poll": (i, [vp, ctypes.POINTER(KpCompletion), i, d]),
        "kp_server_now": (d, [vp]),
        "kp_server_stats_get": (i, [vp, ctypes.POINTER(KpServerStats)]),
        "kp_server_destroy": (None, [vp]),
        "kp_server_last_error": (ctypes.c_char_p, [vp]),
        "kp_assemble_rhs": (i, [vp, vp, vp, i, pd]),
        "kp_field": (i, [vp, vp, vp, i, pd]),
        "kp_plan_set_preconditioner": (i, [vp, i, i, d]),
        "kp_apply_preconditioner": (i, [vp, vp, vp, i]),
        "kp_last_error": (ctypes.c_char_p, []),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    return lib


_lib = _load()


# ------------------------------------------------------- raw entry points ----
def kp_strerror(status):
    return _lib.kp_strerror(int(status)).decode()


def kp_version():
    return _lib.kp_version().decode()


def kp_last_error():
    return _lib.kp_last_error().decode()


def kp_basis_1d(n, bc):
    """Closed-form orthonormal eigenbasis (host): returns (Q, lam), Q[:, c]
    the c-th eigenvector."""
    Q = np.zeros((n, n))
    lam = np.zeros(n)
    rc = _lib.kp_basis_1d(int(n), BC[bc] if isinstance(bc, str) else int(bc),
                          Q.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                          lam.ctypes.data_as(ctypes.POINTER(ctypes.c_double)))
    if rc != KP_OK:
        raise KpError(rc, "kp_basis_1d")
    return Q, lam


def kp_plan_create(nx, ny, nz, bc, prec, max_batch, stream):
    handle = ctypes.c_void_p()
    arr = (ctypes.c_int * 3)(*bc)
    rc = _lib.kp_plan_create(ctypes.byref(handle), nx, ny, nz, arr, prec, max_batch,
                             ctypes.c_void_p(stream))
    return rc, handle


def kp_plan_destroy(handle):
    _lib.kp_plan_destroy(handle)


def kp_plan_workspace_bytes(handle, batch):
    return int(_lib.kp_plan_workspace_bytes(handle, batch))


def kp_plan_resident_bytes(handle):
    return int(_lib.kp_plan_resident_bytes(handle))


def kp_plan_set_workspace(handle, ptr, nbytes):
    return _lib.kp_plan_set_workspace(handle, ctypes.c_void_p(ptr), nbytes)


def kp_plan_set_stream(handle, stream):
    return _lib.kp_plan_set_stream(handle, ctypes.c_void_p(stream))


def kp_apply_laplacian(handle, p_ptr, w_ptr, batch):
    return _lib.kp_apply_laplacian(handle, ctypes.c_void_p(p_ptr), ctypes.c_void_p(w_ptr), batch)


def kp_apply_pinv(handle, r_ptr, z_ptr, batch):
    return _lib.kp_apply_pinv(handle, ctypes.c_void_p(r_ptr), ctypes.c_void_p(z_ptr), batch)


def kp_apply_pinv_noalloc(handle, r_ptr, z_ptr, batch):
    return _lib.kp_apply_pinv_noalloc(handle, ctypes.c_void_p(r_ptr), ctypes.c_void_p(z_ptr),
                                      batch)


def kp_solve(handle, eta_ptr, u_ptr, batch, tol, max_iter, flags, results, hist):
    hp = hist.ctypes.data_as(ctypes.POINTER(ctypes.c_double)) if hist is not None else None
    return _lib.kp_solve(handle, ctypes.c_void_p(eta_ptr), ctypes.c_void_p(u_ptr), batch,
                         float(tol), int(max_iter), int(flags), results, hp)


def kp_solve_async(handle, eta_ptr, u_ptr, batch, tol, max_iter, flags, results, hist):
    """(status, ticket handle); results and hist must stay alive until
    kp_wait has returned."""
    hp = hist.ctypes.data_as(ctypes.POINTER(ctypes.c_double)) if hist is not None else None
    ticket = ctypes.c_void_p()
    rc = _lib.kp_solve_async(handle, ctypes.c_void_p(eta_ptr), ctypes.c_void_p(u_ptr), batch,
                             float(tol), int(max_iter), int(flags), results, hp,
                             ctypes.byref(ticket))
    return rc, ticket


def kp_poll(ticket):
    return _lib.kp_poll(ticket)


def kp_wait(ticket):
    return _lib.kp_wait(ticket)


def kp_plan_set_profiling(handle, enable):
    return _lib.kp_plan_set_profiling(handle, int(enable))


def kp_plan_profile(handle, cls):
    ms = ctypes.c_double()
    cnt = ctypes.c_int64()
    rc = _lib.kp_plan_profile(handle, int(cls), ctypes.byref(ms), ctypes.byref(cnt))
    return rc, ms.value, cnt.value


def kp_plan_profile_reset(handle):
    return _lib.kp_plan_profile_reset(handle)


def kp_kernel_class_name(cls):
    return _lib.kp_kernel_class_name(int(cls)).decode()


def kp_plan_autotune(handle, batch, reps):
    chosen = (ctypes.c_int * 6)()
    rc = _lib.kp_plan_autotune(handle, int(batch), int(reps), chosen)
    return rc, list(chosen)


def kp_plan_time_kernel(handle, cls, batch, flags, reps):
    ms = ctypes.c_double()
    rc = _lib.kp_plan_time_kernel(handle, int(cls), int(batch), int(flags), int(reps),
                                  ctypes.byref(ms))
    return rc, ms.value


def kp_plan_diagnostics(handle, batch, hs, delay):
    out = np.zeros((batch, hs, KP_DIAG_COLUMNS))
    rc = _lib.kp_plan_diagnostics(handle, out.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                  int(batch), int(hs), int(delay))
    return rc, out


def kp_lowrank_table(n, bc_n, q, bc_q, rank):
    """G_r of the low-rank preconditioner as an (q, n) array (host only)."""
    out = np.zeros((q, n))
    code = lambda bc: BC[bc] if isinstance(bc, str) else int(bc)
    rc = _lib.kp_lowrank_table(int(n), code(bc_n), int(q), code(bc_q), int(rank),
                               out.ctypes.data_as(ctypes.POINTER(ctypes.c_double)))
    if rc != KP_OK:
        raise KpError(rc, "kp_lowrank_table")
    return out


def kp_plan_get_tuning(handle):
    cfg = (ctypes.c_int * 6)()
    n = _lib.kp_plan_get_tuning(handle, cfg, 6)
    return n, list(cfg)[: max(n, 0)]


def kp_plan_set_tuning(handle, cfg):
    arr = (ctypes.c_int * len(cfg))(*cfg)
    return _lib.kp_plan_set_tuning(handle, arr, len(cfg))


def kp_plan_graph_count(handle):
    return _lib.kp_plan_graph_count(handle)


def kp_tile_shape(cfg_id, prec):
    """(status, (wn, wm, wc)) of a tile configuration for a precision code."""
    wn, wm, wc = ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
    rc = _lib.kp_tile_shape(int(cfg_id), int(prec), ctypes.byref(wn), ctypes.byref(wm),
                            ctypes.byref(wc))
    return rc, (wn.value, wm.value, wc.value)


def kp_server_create(hbm_budget, workers, max_batch):
    handle = ctypes.c_void_p()
    rc = _lib.kp_server_create(ctypes.byref(handle), int(hbm_budget), int(workers), int(max_batch))
    return rc, handle


def kp_server_submit(handle, req):
    return _lib.kp_server_submit(handle, ctypes.byref(req))


def kp_server_poll(handle, max_n, timeout_s):
    out = (KpCompletion * max_n)()
    n = _lib.kp_server_poll(handle, out, int(max_n), float(timeout_s))
    return n, [out[k].as_dict() for k in range(max(n, 0))]


def kp_server_now(handle):
    return _lib.kp_server_now(handle)


def kp_server_stats_get(handle):
    st = KpServerStats()
    rc = _lib.kp_server_stats_get(handle, ctypes.byref(st))
    return rc, st.as_dict()


def kp_server_destroy(handle):
    _lib.kp_server_destroy(handle)


# ------------------------------------------------------------ torch layer ----
def _torch():
    import torch
    return torch


class Plan:
    """A plan for one grid, boundary-condition triple and precision.

    Grid functions are float64 CUDA tensors shaped (nz, ny, nx) (3D),
    (ny, nx) (2D) or with a leading batch dimension.
    """

    def __init__(self, nx, ny, nz, bcs, prec="f64", max_batch=1, stream=None):
        torch = _torch()
        self.shape = (nz, ny, nx) if nz > 1 else (ny, nx)
        self.N = nx * ny * nz
        self.dims = (nx, ny, nz)
        bcs = tuple(bcs) + ("D",) * (3 - len(bcs))
        self.bcs = bcs
        self.prec = prec
        self.max_batch = max_batch
        if stream is None:
            stream = torch.cuda.current_stream()
        self.stream = stream
        rc, self._h = kp_plan_create(nx, ny, nz, [BC[b] for b in bcs], PREC[prec], max_batch,
                                     stream.cuda_stream)
        if rc != KP_OK:
            raise KpError(rc, "kp_plan_create")

    def close(self):
        if getattr(self, "_h", None):
            kp_plan_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def workspace_bytes(self):
        return kp_plan_workspace_bytes(self._h, self.max_batch)

    @property
    def resident_bytes(self):
        return kp_plan_resident_bytes(self._h)

    def _check(self, t, name):
        torch = _torch()
        if not (t.is_cuda and t.dtype == torch.float64 and t.is_contiguous()):
            raise ValueError(f"{name} must be a contiguous float64 CUDA tensor")
        if t.numel() % self.N:
            raise ValueError(f"{name} size is not a multiple of the grid size")
        return t.numel() // self.N

    def tuning_key(self, batch=1):
        nx, ny, nz = self.dims
        return f"{nx}x{ny}x{nz}:{self.prec}:b{batch}"

    def autotune(self, batch=1, reps=5, cache=None):
        """Times every tile shape for each mode product and keeps the fastest
        (the operator-resident shapes only on axes of at most 128).  With
        `cache` (a path), reuses and records choices in a JSON file."""
        import json
        key = self.tuning_key(batch)
        if cache and os.path.exists(cache):
            with open(cache) as f:
                table = json.load(f)
            if key in table and kp_plan_set_tuning(self._h, table[key]) == KP_OK:
                return table[key]
        rc, chosen = kp_plan_autotune(self._h, batch, reps)
        if rc != KP_OK:
            raise KpError(rc, "kp_plan_autotune")
        n, cfg = kp_plan_get_tuning(self._h)
        if cache:
            table = {}
            if os.path.exists(cache):
                with open(cache) as f:
                    table = json.load(f)
            table[key] = cfg
            with open(cache, "w") as f:
                json.dump(table, f, indent=1, sort_keys=True)
        return cfg

    @property
    def tuning(self):
        return kp_plan_get_tuning(self._h)[1]

    @tuning.setter
    def tuning(self, cfg):
        rc = kp_plan_set_tuning(self._h, list(cfg))
        if rc != KP_OK:
            raise KpError(rc, "kp_plan_set_tuning")

    def set_profiling(self, enable=True):
        rc = kp_plan_set_profiling(self._h, enable)
        if rc != KP_OK:
            raise KpError(rc, "kp_plan_set_profiling")

    def time_kernel(self, cls, batch=1, flags=0, reps=100):
        """Average milliseconds of one launch of a kernel class (name or
        number), `reps` launches back to back on workspace data; the
        one-kernel 2D solve ("small_solve") is timed on the arguments of the
        plan's last solve that took it (kp_plan_time_kernel)."""
        if isinstance(cls, str):
            names = [kp_kernel_class_name(c) for c in range(KERNEL_CLASSES)]
            cls = names.index(cls)
        rc, ms = kp_plan_time_kernel(self._h, cls, batch, flags, reps)
        if rc != KP_OK:
            raise KpError(rc, "kp_plan_time_kernel")
        return ms

    def profile(self):
        """{class name: (total_ms, launches)} accumulated since the last reset."""
        out = {}
        for c in range(KERNEL_CLASSES):
            rc, ms, cnt = kp_plan_profile(self._h, c)
            if rc != KP_OK:
                raise KpError(rc, "kp_plan_profile")
            out[kp_kernel_class_name(c)] = (ms, cnt)
        return out

    def profile_reset(self):
        rc = kp_plan_profile_reset(self._h)
        if rc != KP_OK:
            raise KpError(rc, "kp_plan_profile_reset")

    def apply_laplacian(self, P, out=None):
        batch = self._check(P, "P")
        W = out if out is not None else _torch().empty_like(P)
        rc = kp_apply_laplacian(self._h, P.data_ptr(), W.data_ptr(), batch)
        if rc != KP_OK:
            raise KpError(rc, "kp_apply_laplacian")
        return W

    def apply_pinv(self, R, out=None):
        batch = self._check(R, "R")
        Z = out if out is not None else _torch().empty_like(R)
        rc = kp_apply_pinv(self._h, R.data_ptr(), Z.data_ptr(), batch)
        if rc != KP_OK:
            raise KpError(rc, "kp_apply_pinv")
        return Z

    def _faces(self, faces, batch):
        if faces is None:
            return None, None
        dim = 3 if self.dims[2] > 1 else 2
        f = np.ascontiguousarray(np.broadcast_to(np.asarray(faces, dtype=np.float64),
                                                 (batch, dim, 2)))
        return f, f.ctypes.data_as(ctypes.POINTER(ctypes.c_double))

    def set_preconditioner(self, kind="pinv", steps=3, omega=1.3):
        """'pinv' (default), 'jacobi' with p = steps and omega, or 'lowrank'
        (2D) with Kronecker rank = steps."""
        code = {"pinv": 0, "jacobi": 1, "lowrank": 2}[kind]
        rc = _lib.kp_plan_set_preconditioner(self._h, code, int(steps), float(omega))
        if rc != KP_OK:
            raise KpError(rc, "kp_plan_set_preconditioner")

    def apply_preconditioner(self, R, out=None):
        batch = self._check(R, "R")
        Z = out if out is not None else _torch().empty_like(R)
        rc = _lib.kp_apply_preconditioner(self._h, R.data_ptr(), Z.data_ptr(), batch)
        if rc != KP_OK:
            raise KpError(rc, "kp_apply_preconditioner")
        return Z

    def assemble_rhs(self, eta, faces=None, out=None):
        """eta plus the boundary-data update of kp_assemble_rhs; faces is
        (dim, 2) or (batch, dim, 2): [axis][beginning, end]."""
        batch = self._check(eta, "eta")
        rhs = out if out is not None else _torch().empty_like(eta)
        f, fp = self._faces(faces, batch)
        rc = _lib.kp_assemble_rhs(self._h, eta.data_ptr(), rhs.data_ptr(), batch, fp)
        if rc != KP_OK:
            raise KpError(rc, "kp_assemble_rhs")
        return rhs

    def field(self, u, faces=None, out=None):
        """eps = -grad u, shaped (dim,) + grid (with a leading batch axis for
        a batch)."""
        torch = _torch()
        batch = self._check(u, "u")
        dim = 3 if self.dims[2] > 1 else 2
        shape = ((batch,) if u.dim() > len(self.shape) else ()) + (dim,) + self.shape
        eps = out if out is not None else torch.empty(shape, dtype=torch.float64, device=u.device)
        f, fp = self._faces(faces, batch)
        rc = _lib.kp_field(self._h, u.data_ptr(), eps.data_ptr(), batch, fp)
        if rc != KP_OK:
            raise KpError(rc, "kp_field")
        return eps

    def solve(self, eta, tol=1e-10, max_iter=50, flags=0, out=None, raise_on_error=True):
        """Returns (u, results, history, status); results is a list of dicts,
        history a (batch, max_iter+1) numpy array of ||R_s|| / ||eta_c||.
        With KP_FLAG_WARM_START, `out` holds U_0 on entry."""
        batch = self._check(eta, "eta")
        if (flags & KP_FLAG_WARM_START) and out is None:
            raise ValueError("a warm start takes U_0 in `out`")
        u = out if out is not None else _torch().empty_like(eta)
        results = (KpResult * batch)()
        hist = np.zeros((batch, max_iter + 1))
        rc = kp_solve(self._h, eta.data_ptr(), u.data_ptr(), batch, tol, max_iter, flags,
                      results, hist)
        self._last_shape = (batch, max_iter + 1)
        if rc < 0 and raise_on_error:
            raise KpError(rc, "kp_solve")
        return u, [r.as_dict() for r in results], hist, rc

    def solve_async(self, eta, tol=1e-10, max_iter=50, flags=0, out=None):
        """Enqueues the solve and returns a Ticket at once (kp_solve_async);
        ticket.poll() is True once it has finished, ticket.wait() returns
        (u, results, history, status) as solve() does."""
        batch = self._check(eta, "eta")
        if (flags & KP_FLAG_WARM_START) and out is None:
            raise ValueError("a warm start takes U_0 in `out`")
        u = out if out is not None else _torch().empty_like(eta)
        results = (KpResult * batch)()
        hist = np.zeros((batch, max_iter + 1))
        rc, th = kp_solve_async(self._h, eta.data_ptr(), u.data_ptr(), batch, tol, max_iter,
                                flags, results, hist)
        if rc != KP_OK:
            raise KpError(rc, "kp_solve_async")
        self._last_shape = (batch, max_iter + 1)
        return Ticket(th, eta, u, results, hist)

    def diagnostics(self, delay=4):
        """Descriptors of every iterate of the last solve, which must have
        used KP_FLAG_DIAGNOSTICS: a (batch, max_iter+1, 7) array with the
        columns DIAG_COLUMNS (NaN after a right-hand side's last iterate)."""
        batch, hs = getattr(self, "_last_shape", (0, 0))
        rc, out = kp_plan_diagnostics(self._h, max(batch, 1), max(hs, 1), delay)
        if rc != KP_OK:
            raise KpError(rc, "kp_plan_diagnostics")
        return out


class Ticket:
    """A solve in flight (kp_solve_async).  Keeps eta, u and the result
    arrays alive until wait() has returned."""

    def __init__(self, handle, eta, u, results, hist):
        self._h = handle
        self._keep = (eta, u, results, hist)
        self._out = None

    def poll(self):
        """True once the solve has finished; each call that finds the device
        idle also enqueues the next iteration of a solve that continues."""
        if self._h is None:
            return True
        rc = kp_poll(self._h)
        if rc < 0:
            raise KpError(rc, "kp_poll")
        return rc == 1

    def wait(self, raise_on_error=True):
        """Blocks until the solve has finished; (u, results, history, status)."""
        if self._h is not None:
            rc = kp_wait(self._h)
            self._h = None
            eta, u, results, hist = self._keep
            self._out = (u, [r.as_dict() for r in results], hist, rc)
        if self._out[3] < 0 and raise_on_error:
            raise KpError(self._out[3], "kp_wait")
        return self._out

    def __del__(self):
        try:
            if self._h is not None:
                kp_wait(self._h)
                self._h = None
        except Exception:
            pass


class Server:
    """Request server (kp_server_*): plan cache under an HBM budget, worker
    threads with their own streams, batching of queued requests that share a
    plan.  eta / u are float64 CUDA tensors (device requests) or numpy arrays
    (host requests) shaped (nz, ny, nx) or (ny, nx); they are kept alive here
    until their completion has been polled."""

    def __init__(self, hbm_budget=0, workers=4, max_batch=8):
        _torch().cuda.current_device()
        rc, self._h = kp_server_create(hbm_budget, workers, max_batch)
        if rc != KP_OK:
            raise KpError(rc, "kp_server_create")
        self._live = {}

    def submit(self, req_id, eta, bcs, tol=1e-10, prec="f32", max_iter=50, flags=0, u=None):
        torch = _torch()
        shape = tuple(eta.shape)
        if len(shape) == 3:
            nz, ny, nx = shape
        elif len(shape) == 2:
            (ny, nx), nz = shape, 1
        else:
            raise ValueError("eta must be (nz, ny, nx) or (ny, nx)")
        on_dev = isinstance(eta, torch.Tensor)
        if on_dev:
            if eta.dtype != torch.float64 or not eta.is_cuda or not eta.is_contiguous():
                raise ValueError("device eta must be a contiguous float64 CUDA tensor")
            if u is not None and (tuple(u.shape) != shape or u.dtype != torch.float64
                                  or not u.is_cuda or not u.is_contiguous()):
                raise ValueError("u must match eta")
            eptr, uptr = eta.data_ptr(), (u.data_ptr() if u is not None else None)
        else:
            eta = np.ascontiguousarray(eta, dtype=np.float64)
            if u is not None and (u.shape != shape or u.dtype != np.float64
                                  or not u.flags["C_CONTIGUOUS"]):
                raise ValueError("u must match eta")
            eptr, uptr = eta.ctypes.data, (u.ctypes.data if u is not None else None)
        bcs = tuple(bcs) + ("D",) * (3 - len(bcs))
        req = KpRequest(id=int(req_id), nx=nx, ny=ny, nz=nz,
                        bc=(ctypes.c_int * 3)(*[BC[b] for b in bcs]), prec=PREC[prec],
                        tol=float(tol), max_iter=int(max_iter), flags=int(flags),
                        mem=KP_MEM_DEVICE if on_dev else KP_MEM_HOST, eta=eptr, u=uptr)
        self._live[int(req_id)] = (eta, u)
        rc = kp_server_submit(self._h, req)
        if rc != KP_OK:
            self._live.pop(int(req_id), None)
            raise KpError(rc, "kp_server_submit")

    def poll(self, max_n=256, timeout=0.1):
        n, done = kp_server_poll(self._h, max_n, timeout)
        if n < 0:
            raise KpError(n, "kp_server_poll")
        for c in done:
            self._live.pop(c["id"], None)
        return done

    def now(self):
        return kp_server_now(self._h)

    def last_error(self):
        return _lib.kp_server_last_error(self._h).decode()

    def stats(self):
        rc, st = kp_server_stats_get(self._h)
        if rc != KP_OK:
            raise KpError(rc, "kp_server_stats_get")
        return st

    def close(self):
        if getattr(self, "_h", None):
            kp_server_destroy(self._h)
            self._h = None
            self._live.clear()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
