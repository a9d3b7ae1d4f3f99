"""ctypes binding of libvemg.so (argument marshalling only).

Device vectors are torch.float64 CUDA tensors (HIP on ROCm) passed by
data_ptr(); the handle runs on the caller's current torch stream.  Nothing
here computes: a missing library raises at once.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB = None

STATUS = {0: "ok", 1: "max_iter", 2: "floor", -1: "invalid_arg", -2: "mesh", -3: "projection",
          -4: "oom", -5: "device", -6: "breakdown", -7: "state"}
OP_A, OP_PRECOND, OP_ET, OP_E, OP_VCYCLE_S, OP_VCYCLE_ABAR, OP_GS_FWD, OP_GS_COARSE, OP_COARSEST = range(9)
_PC = {"vl_as": 0, "vl_sor": 1, "jacobi": 2, "none": 3, "vl_add": 4, "sa": 5}
_TOP = {"pinned": 0, "N": 0, "dirichlet": 1, "D": 1, "robin": 2, "R": 2}
_PREC = {"fp64": 0, "mixed": 1, "mixed_ir": 1, "mixed_pc": 2}
_EXTRAP = {"projection": 0, "sspai": 1}


class VemgError(RuntimeError):
    def __init__(self, status, msg=""):
        super().__init__(f"vemg status {status} ({STATUS.get(status, '?')}): {msg}")
        self.status = status


class Options(C.Structure):
    _fields_ = [("top_bc", C.c_int), ("pin_node", C.c_int64), ("pc", C.c_int),
                ("theta", C.c_double), ("prolong_omega", C.c_double), ("max_levels", C.c_int),
                ("coarse_max", C.c_int64), ("poll_every", C.c_int), ("max_restarts", C.c_int),
                ("use_graphs", C.c_int), ("precision", C.c_int), ("inner_rtol", C.c_double),
                ("max_outer", C.c_int), ("robin_alpha", C.c_double), ("extrapolation", C.c_int)]


class Info(C.Structure):
    _fields_ = [("n_nodes", C.c_int64), ("n", C.c_int64), ("n_top", C.c_int64), ("pin_node", C.c_int64),
                ("nnz_offdiag", C.c_int64), ("s_levels", C.c_int), ("abar_levels", C.c_int),
                ("s_rows", C.c_int64 * 16), ("abar_rows", C.c_int64 * 16),
                ("s_nnz", C.c_int64 * 16), ("abar_nnz", C.c_int64 * 16),
                ("p_nnz_s", C.c_int64 * 16), ("p_nnz_abar", C.c_int64 * 16),
                ("e_nnz", C.c_int64), ("fine_colours_top", C.c_int), ("fine_colours_bar", C.c_int),
                ("device_bytes", C.c_size_t)]


class ServerStats(C.Structure):
    _fields_ = [("requests_done", C.c_int64), ("columns_done", C.c_int64), ("requests_queued", C.c_int64),
                ("p50_ms", C.c_double), ("p99_ms", C.c_double), ("mean_ms", C.c_double), ("max_ms", C.c_double),
                ("solves_per_s", C.c_double), ("busy_s", C.c_double), ("mean_slot_occupancy", C.c_double),
                ("chunks", C.c_int64), ("uploads", C.c_int64), ("evictions", C.c_int64),
                ("resident_bytes", C.c_size_t), ("budget_bytes", C.c_size_t)]


def library_path():
    return os.path.join(_HERE, "libvemg.so")


def load_library():
    global _LIB
    if _LIB is not None:
        return _LIB
    path = library_path()
    if not os.path.exists(path):
        raise ImportError(f"{path} is missing: build it with paper_0912_1976_amd/build.py")
    lib = C.CDLL(path)
    P, I64, I32, D = C.c_void_p, C.c_int64, C.c_int, C.c_double
    lib.vemg_default_options.argtypes = [C.POINTER(Options)]
    lib.vemg_default_options.restype = None
    lib.vemg_create.argtypes = [C.POINTER(Options), I32, P, C.POINTER(P)]
    lib.vemg_setup.argtypes = [P, I64, P, I64, P, P]
    lib.vemg_rhs.argtypes = [P, P, P]
    lib.vemg_matvec.argtypes = [P, P, P]
    lib.vemg_matvec_noalloc.argtypes = [P, P, P]
    lib.vemg_solve.argtypes = [P, I32, P, P, D, I32, P, P]
    lib.vemg_apply.argtypes = [P, I32, P, P]
    lib.vemg_get_info.argtypes = [P, C.POINTER(Info)]
    lib.vemg_footprint.argtypes = [P, I32, C.POINTER(C.c_size_t)]
    lib.vemg_set_preconditioner.argtypes = [P, I32]
    lib.vemg_set_precision.argtypes = [P, I32]
    lib.vemg_time_op.argtypes = [P, I32, I32, I32, C.POINTER(C.c_double), C.POINTER(C.c_int)]
    lib.vemg_export.argtypes = [P, C.c_char_p, P, C.POINTER(C.c_size_t)]
    lib.vemg_destroy.argtypes = [P]
    lib.vemg_status_string.argtypes = [I32]
    lib.vemg_status_string.restype = C.c_char_p
    lib.vemg_last_error.argtypes = [P]
    lib.vemg_last_error.restype = C.c_char_p
    U64 = C.c_uint64
    lib.vemg_server_create.argtypes = [I32, C.c_size_t, C.POINTER(Options), C.POINTER(P)]
    lib.vemg_server_add_mesh.argtypes = [P, I64, P, I64, P, P, C.POINTER(I32)]
    lib.vemg_server_rhs.argtypes = [P, I32, P, P]
    lib.vemg_server_footprint.argtypes = [P, I32, I32, C.POINTER(C.c_size_t)]
    lib.vemg_server_submit.argtypes = [P, I32, I32, P, P, D, I32, C.POINTER(U64)]
    lib.vemg_server_poll.argtypes = [P, C.POINTER(U64), I32, C.POINTER(I32)]
    lib.vemg_server_wait.argtypes = [P, U64, D]
    lib.vemg_server_result.argtypes = [P, U64, C.POINTER(I32), P, P, C.POINTER(D)]
    lib.vemg_server_get_stats.argtypes = [P, C.POINTER(ServerStats)]
    lib.vemg_server_destroy.argtypes = [P]
    lib.vemg_server_set_precision.argtypes = [P, I32]
    lib.vemg_server_last_error.argtypes = [P]
    lib.vemg_server_last_error.restype = C.c_char_p
    for f in ("vemg_server_create", "vemg_server_add_mesh", "vemg_server_rhs", "vemg_server_footprint",
              "vemg_server_submit",
              "vemg_server_poll", "vemg_server_wait", "vemg_server_result", "vemg_server_get_stats",
              "vemg_server_destroy", "vemg_server_set_precision"):
        getattr(lib, f).restype = I32
    for f in ("vemg_create", "vemg_setup", "vemg_rhs", "vemg_matvec", "vemg_matvec_noalloc", "vemg_solve", "vemg_apply",
              "vemg_get_info", "vemg_footprint", "vemg_export", "vemg_destroy", "vemg_time_op"):
        getattr(lib, f).restype = I32
    _LIB = lib
    return lib


def _ptr(t):
    return C.c_void_p(t.data_ptr())


class Solver:
    """One mesh, set up once, solved many times.

    device: HIP ordinal, or -1 for a host-only setup (inspection, no solves).
    """

    def __init__(self, xyz, tets, top, *, top_bc="pinned", pc="vl_as", device=0, pin_node=-1,
                 use_graphs=True, poll_every=8, coarse_max=8192, max_levels=10, max_restarts=5,
                 precision="fp64", inner_rtol=1e-4, max_outer=30, robin_alpha=0.0,
                 extrapolation="projection"):
        self._lib = load_library()
        opt = Options()
        self._lib.vemg_default_options(C.byref(opt))
        opt.top_bc = _TOP[top_bc]
        opt.robin_alpha = robin_alpha
        opt.extrapolation = _EXTRAP[extrapolation]
        opt.pc = _PC[pc]
        opt.pin_node = pin_node
        opt.use_graphs = int(bool(use_graphs))
        opt.poll_every = poll_every
        opt.coarse_max = coarse_max
        opt.max_levels = max_levels
        opt.max_restarts = max_restarts
        opt.precision = _PREC[precision]
        opt.inner_rtol = inner_rtol
        opt.max_outer = max_outer
        self.precision = precision
        self.device = device
        stream = None
        if device >= 0:
            import torch
            self._torch = torch
            self.dev = torch.device("cuda", device)
            stream = C.c_void_p(torch.cuda.current_stream(self.dev).cuda_stream)
        h = C.c_void_p()
        self._check(self._lib.vemg_create(C.byref(opt), device, stream, C.byref(h)), None)
        self._h = h
        xyz = np.ascontiguousarray(xyz, dtype=np.float64)
        tets = np.ascontiguousarray(tets, dtype=np.int64)
        top = np.ascontiguousarray(top, dtype=np.uint8)
        self.n_nodes = xyz.shape[0]
        self._check(self._lib.vemg_setup(h, self.n_nodes, xyz.ctypes.data, tets.shape[0], tets.ctypes.data,
                                         top.ctypes.data), h)

    def _check(self, st, h):
        if st < 0:
            msg = self._lib.vemg_last_error(h).decode() if h else ""
            raise VemgError(st, msg)
        return st

    def close(self):
        if getattr(self, "_h", None):
            self._lib.vemg_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ---------------------------------------------------------------- info
    def set_preconditioner(self, pc):
        """Switch the preconditioner ('vl_as', 'vl_sor', 'vl_add', 'jacobi',
        'none') without repeating the setup."""
        self._check(self._lib.vemg_set_preconditioner(self._h, _PC[pc]), self._h)

    def set_precision(self, precision):
        """Switch between 'fp64', 'mixed_ir' and 'mixed_pc' for later solves."""
        self._check(self._lib.vemg_set_precision(self._h, _PREC[precision]), self._h)

    def info(self):
        inf = Info()
        self._check(self._lib.vemg_get_info(self._h, C.byref(inf)), self._h)
        out = {k: getattr(inf, k) for k, _ in Info._fields_}
        for k in ("s_rows", "abar_rows", "s_nnz", "abar_nnz", "p_nnz_s", "p_nnz_abar"):
            out[k] = list(out[k])
        out["s_rows"] = out["s_rows"][: inf.s_levels]
        out["abar_rows"] = out["abar_rows"][: inf.abar_levels]
        for k, nl in (("s_nnz", inf.s_levels), ("p_nnz_s", inf.s_levels), ("abar_nnz", inf.abar_levels),
                      ("p_nnz_abar", inf.abar_levels)):
            out[k] = out[k][:nl]
        return out

    def footprint(self, nrhs=0):
        """Device bytes for a solve of nrhs right-hand sides (the handle's
        resident memory plus 2 * nrhs * n_nodes doubles for b and x)."""
        nb = C.c_size_t(0)
        self._check(self._lib.vemg_footprint(self._h, nrhs, C.byref(nb)), self._h)
        return nb.value

    def export(self, name, dtype):
        nb = C.c_size_t(0)
        self._check(self._lib.vemg_export(self._h, name.encode(), None, C.byref(nb)), self._h)
        arr = np.empty(nb.value // np.dtype(dtype).itemsize, dtype=dtype)
        self._check(self._lib.vemg_export(self._h, name.encode(), arr.ctypes.data, C.byref(nb)), self._h)
        return arr

    # ---------------------------------------------------------------- compute
    def rhs(self, f):
        f = np.ascontiguousarray(f, dtype=np.float64)
        b = np.empty_like(f)
        self._check(self._lib.vemg_rhs(self._h, f.ctypes.data, b.ctypes.data), self._h)
        return b

    def _dev(self, a):
        t = self._torch
        if not isinstance(a, t.Tensor):
            a = t.as_tensor(np.asarray(a, dtype=np.float64))
        return a.to(device=self.dev, dtype=t.float64).contiguous()

    def matvec(self, x):
        x = self._dev(x)
        y = self._torch.empty_like(x)
        self._check(self._lib.vemg_matvec(self._h, _ptr(x), _ptr(y)), self._h)
        return y

    def solve(self, b, rtol=1e-8, max_iter=1000):
        """b: [n_nodes] or [nrhs, n_nodes].  Returns (x, iters, relres, status)."""
        b = self._dev(b)
        nrhs = 1 if b.dim() == 1 else b.shape[0]
        x = self._torch.empty_like(b)
        its = (C.c_int * nrhs)()
        rel = (C.c_double * nrhs)()
        st = self._check(self._lib.vemg_solve(self._h, nrhs, _ptr(b), _ptr(x), rtol, max_iter, its, rel), self._h)
        return x, list(its), list(rel), st

    def time_op(self, op, reps=20, nrhs=1):
        """(average ms per application, kernel launches per application)."""
        ms = C.c_double(0.0)
        nl = C.c_int(0)
        self._check(self._lib.vemg_time_op(self._h, op, nrhs, reps, C.byref(ms), C.byref(nl)), self._h)
        return ms.value, nl.value

    def apply(self, op, v, out_len):
        v = self._dev(v)
        out = self._torch.empty(out_len, dtype=self._torch.float64, device=self.dev)
        self._check(self._lib.vemg_apply(self._h, op, _ptr(v), _ptr(out)), self._h)
        return out


class Server:
    """Continuous-batching solve server over several resident meshes.

    Device buffers of every submitted request are kept alive here until the
    request is collected with result()."""

    def __init__(self, *, device=0, hbm_budget=0, top_bc="pinned", pc="vl_as", precision="mixed_pc",
                 poll_every=8, coarse_max=8192, max_restarts=5, robin_alpha=0.0, extrapolation="projection"):
        import torch
        self._torch = torch
        self._lib = load_library()
        opt = Options()
        self._lib.vemg_default_options(C.byref(opt))
        opt.top_bc = _TOP[top_bc]
        opt.robin_alpha = robin_alpha
        opt.extrapolation = _EXTRAP[extrapolation]
        opt.pc = _PC[pc]
        opt.precision = _PREC[precision]
        opt.poll_every = poll_every
        opt.coarse_max = coarse_max
        opt.max_restarts = max_restarts
        self.dev = torch.device("cuda", device)
        h = C.c_void_p()
        self._check(self._lib.vemg_server_create(device, hbm_budget, C.byref(opt), C.byref(h)))
        self._h = h
        self._live = {}
        self.n_nodes = []

    def _check(self, st):
        if st < 0:
            msg = self._lib.vemg_server_last_error(self._h).decode() if getattr(self, "_h", None) else ""
            raise VemgError(st, msg)
        return st

    def add_mesh(self, xyz, tets, top):
        xyz = np.ascontiguousarray(xyz, dtype=np.float64)
        tets = np.ascontiguousarray(tets, dtype=np.int64)
        top = np.ascontiguousarray(top, dtype=np.uint8)
        mid = C.c_int(0)
        self._check(self._lib.vemg_server_add_mesh(self._h, xyz.shape[0], xyz.ctypes.data, tets.shape[0],
                                                   tets.ctypes.data, top.ctypes.data, C.byref(mid)))
        self.n_nodes.append(xyz.shape[0])
        return mid.value

    def rhs(self, mesh_id, f):
        f = np.ascontiguousarray(f, dtype=np.float64)
        b = np.empty_like(f)
        self._check(self._lib.vemg_server_rhs(self._h, mesh_id, f.ctypes.data, b.ctypes.data))
        return b

    def footprint(self, mesh_id, nrhs=0):
        nb = C.c_size_t(0)
        self._check(self._lib.vemg_server_footprint(self._h, mesh_id, nrhs, C.byref(nb)))
        return nb.value

    def submit(self, mesh_id, b, rtol=1e-8, max_iter=5000):
        """b: CUDA float64 tensor [nrhs, n_nodes] (written and synchronised)."""
        torch = self._torch
        b = b.to(device=self.dev, dtype=torch.float64).contiguous()
        if b.dim() == 1:
            b = b[None]
        x = torch.empty_like(b)
        torch.cuda.synchronize(self.dev)
        rid = C.c_uint64(0)
        self._check(self._lib.vemg_server_submit(self._h, mesh_id, b.shape[0], _ptr(b), _ptr(x), rtol, max_iter,
                                                 C.byref(rid)))
        self._live[rid.value] = (b, x)
        return rid.value

    def poll(self, cap=1024):
        ids = (C.c_uint64 * cap)()
        n = C.c_int(0)
        self._check(self._lib.vemg_server_poll(self._h, ids, cap, C.byref(n)))
        return [ids[i] for i in range(n.value)]

    def wait(self, rid, timeout=0.0):
        self._check(self._lib.vemg_server_wait(self._h, rid, timeout))

    def result(self, rid):
        """(x tensor [nrhs, n_nodes], status, iters, relres, latency_ms); releases the request.
        Raises (keeping the request's buffers alive) while it is not complete."""
        b, x = self._live[rid]
        nrhs = b.shape[0]
        st = C.c_int(0)
        its = (C.c_int * nrhs)()
        rel = (C.c_double * nrhs)()
        lat = C.c_double(0.0)
        self._check(self._lib.vemg_server_result(self._h, rid, C.byref(st), its, rel, C.byref(lat)))
        # the library has reported the request done: its kernels no longer use b or x
        del self._live[rid]
        return x, st.value, list(its), list(rel), lat.value

    def set_precision(self, precision):
        self._check(self._lib.vemg_server_set_precision(self._h, _PREC[precision]))

    def stats(self):
        s = ServerStats()
        self._check(self._lib.vemg_server_get_stats(self._h, C.byref(s)))
        return {k: getattr(s, k) for k, _ in ServerStats._fields_}

    def close(self):
        if getattr(self, "_h", None):
            self._lib.vemg_server_destroy(self._h)
            self._h = None
            self._live.clear()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
