"""ctypes binding of the C ABI in include/bddc.h (argument marshalling only).

Every function of the C ABI is exposed under the same name; ``BDDC`` is a
small convenience wrapper around one context.  Vectors handed to apply /
solve are torch tensors in float64 on the context's GPU: the binding passes
their device pointers and torch's current stream, so the library's kernels are
ordered after whatever produced the inputs.  There is no fallback: if the
library is missing or the GPU is absent the calls raise.
"""
from __future__ import annotations

import atexit
import ctypes as C
import os
import weakref

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libbddc_mi355x.so")

STATUS = {0: "BDDC_OK", 1: "BDDC_ERR_ARG", 2: "BDDC_ERR_STATE", 3: "BDDC_ERR_OOM",
          4: "BDDC_ERR_NOT_SPD", 5: "BDDC_ERR_SINGULAR_COARSE", 6: "BDDC_ERR_NO_CONVERGENCE",
          7: "BDDC_ERR_INSUFFICIENT_CORNERS", 8: "BDDC_ERR_DEVICE"}

MODES = {"c": 0, "ce": 1, "cef": 2, "all": 3}


class BddcError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{STATUS.get(code, code)}: {msg}")
        self.code = code


ALLOC_FN = C.CFUNCTYPE(C.c_void_p, C.c_size_t, C.c_void_p)
FREE_FN = C.CFUNCTYPE(None, C.c_void_p, C.c_void_p)


class bddc_options(C.Structure):
    _fields_ = [("device", C.c_int), ("hip_stream", C.c_void_p), ("factor_precision", C.c_int),
                ("alloc", ALLOC_FN), ("free", FREE_FN), ("alloc_user", C.c_void_p),
                ("verbose", C.c_int), ("autotune", C.c_int),
                ("per_substructure_launches", C.c_int), ("chol_launch", C.c_int)]


class bddc_mesh(C.Structure):
    _fields_ = [("kind", C.c_int), ("n_nodes", C.c_int64), ("xyz", C.POINTER(C.c_double)),
                ("n_elems", C.c_int64), ("hex8", C.POINTER(C.c_int64)),
                ("coef", C.POINTER(C.c_double)), ("nu", C.c_double),
                ("dirichlet", C.POINTER(C.c_uint8))]


class bddc_partition(C.Structure):
    _fields_ = [("n_sub", C.c_int32), ("elem_sub", C.POINTER(C.c_int32))]


class bddc_constraints(C.Structure):
    _fields_ = [("mode", C.c_int), ("augment_corners", C.c_int), ("qr_drop_tol", C.c_double),
                ("adaptive_edges", C.c_int)]


class bddc_pcg_params(C.Structure):
    _fields_ = [("rtol", C.c_double), ("maxit", C.c_int)]


class bddc_pcg_info(C.Structure):
    _fields_ = [("iters", C.c_int), ("converged", C.c_int), ("relres", C.c_double),
                ("kappa", C.c_double), ("lmin", C.c_double), ("lmax", C.c_double),
                ("seconds", C.c_double), ("true_relres", C.c_double), ("refinements", C.c_int),
                ("refine_iters", C.c_int), ("residual_floor", C.c_double)]


class bddc_adapt_info(C.Structure):
    _fields_ = [("omega", C.c_double), ("nc", C.c_int64), ("n_added", C.c_int64),
                ("n_pairs", C.c_int64), ("lobpcg_iters", C.c_int64), ("unconverged", C.c_int64),
                ("seconds", C.c_double), ("n_added_edge", C.c_int64)]


class bddc_info(C.Structure):
    _fields_ = [("n_glob", C.c_int64), ("n_sub", C.c_int64), ("n_corners", C.c_int64),
                ("n_edges", C.c_int64), ("n_faces", C.c_int64), ("nc", C.c_int64),
                ("n_coarse", C.c_int64), ("n_iface_total", C.c_int64),
                ("max_interior", C.c_int64), ("max_iface", C.c_int64),
                ("factor_flops", C.c_double), ("factor_seconds", C.c_double),
                ("apply_bytes", C.c_double), ("pcg_iter_bytes", C.c_double),
                ("device_bytes", C.c_size_t), ("autotune_entries", C.c_int64),
                ("fp32_fallbacks", C.c_int64)]


class bddc_server_options(C.Structure):
    _fields_ = [("device", C.c_int), ("factor_precision", C.c_int), ("max_active", C.c_int),
                ("hbm_budget_bytes", C.c_double), ("resident_bytes", C.c_double)]


class bddc_request_info(C.Structure):
    _fields_ = [("id", C.c_int64), ("state", C.c_int), ("status", C.c_int), ("submit_s", C.c_double),
                ("start_s", C.c_double), ("done_s", C.c_double), ("footprint_bytes", C.c_double),
                ("n_glob", C.c_int64), ("omega", C.c_double), ("nc", C.c_int64),
                ("pcg", bddc_pcg_info), ("error", C.c_char * 160), ("reused", C.c_int),
                ("batch", C.c_int)]


class bddc_kernel_stat(C.Structure):
    _fields_ = [("name", C.c_char * 32), ("ms", C.c_double), ("launches", C.c_int64),
                ("bytes", C.c_double), ("flops", C.c_double)]


SYMBOLS = ["bddc_create", "bddc_setup", "bddc_adapt", "bddc_adapt_count", "bddc_factor",
           "bddc_apply", "bddc_apply_noalloc", "bddc_pcg_solve", "bddc_get_info",
           "bddc_get_face_rows",
           "bddc_get_edge_rows", "bddc_get_face_eigs",
           "bddc_pcg_history", "bddc_get_substructure", "bddc_set_timing", "bddc_get_timing",
           "bddc_server_create", "bddc_server_submit", "bddc_server_wait", "bddc_server_query",
           "bddc_server_release", "bddc_server_destroy", "bddc_last_error", "bddc_destroy"]
# the last entries have their own return types
_VOID = ("bddc_server_destroy", "bddc_destroy")

_lib = None
_live = weakref.WeakSet()


@atexit.register
def _close_all():
    # free device memory through torch before torch itself shuts down
    for b in list(_live):
        try:
            b.close()
        except Exception:
            pass


def load(path: str = LIB_PATH):
    """Load the shared library and declare the C signatures."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"{path} is missing: build it with python -m paper_0910_5863_amd.build")
    L = C.CDLL(path)
    P = C.c_void_p
    L.bddc_create.argtypes = [C.POINTER(bddc_options), C.POINTER(P)]
    L.bddc_setup.argtypes = [P, C.POINTER(bddc_mesh), C.POINTER(bddc_partition),
                             C.POINTER(bddc_constraints)]
    L.bddc_adapt.argtypes = [P, C.c_double, C.POINTER(bddc_adapt_info)]
    L.bddc_adapt_count.argtypes = [P, C.c_int, C.POINTER(bddc_adapt_info)]
    L.bddc_factor.argtypes = [P]
    L.bddc_apply.argtypes = [P, C.c_int, P, C.c_int64, P, C.c_int64]
    L.bddc_pcg_solve.argtypes = [P, C.c_int, P, C.c_int64, P, C.c_int64,
                                 C.POINTER(bddc_pcg_params), C.POINTER(bddc_pcg_info)]
    L.bddc_get_info.argtypes = [P, C.POINTER(bddc_info)]
    L.bddc_get_face_rows.argtypes = [P, C.c_int64, C.c_int64, C.POINTER(C.c_double),
                                     C.POINTER(C.c_int64), C.POINTER(C.c_int64),
                                     C.POINTER(C.c_int64), C.POINTER(C.c_int32)]
    L.bddc_get_edge_rows.argtypes = [P, C.c_int64, C.c_int64, C.POINTER(C.c_double),
                                     C.POINTER(C.c_int64), C.POINTER(C.c_int64),
                                     C.POINTER(C.c_int64)]
    L.bddc_get_face_eigs.argtypes = [P, C.c_int64, C.c_int64, C.POINTER(C.c_double),
                                     C.POINTER(C.c_int64)]
    L.bddc_pcg_history.argtypes = [P, C.c_int64, C.POINTER(C.c_double), C.POINTER(C.c_int64)]
    L.bddc_get_substructure.argtypes = [P, C.c_int32, C.POINTER(C.c_int64), C.POINTER(C.c_int64),
                                        C.POINTER(C.c_int64), C.POINTER(C.c_int64),
                                        C.POINTER(C.c_int64), C.POINTER(C.c_int32),
                                        C.POINTER(C.c_double), C.POINTER(C.c_double)]
    L.bddc_set_timing.argtypes = [P, C.c_int]
    L.bddc_get_timing.argtypes = [P, C.c_int, C.POINTER(bddc_kernel_stat), C.POINTER(C.c_int)]
    L.bddc_last_error.argtypes = [P]
    L.bddc_last_error.restype = C.c_char_p
    L.bddc_destroy.argtypes = [P]
    L.bddc_server_create.argtypes = [C.POINTER(bddc_server_options), C.POINTER(P)]
    L.bddc_server_submit.argtypes = [P, C.POINTER(bddc_mesh), C.POINTER(bddc_partition),
                                     C.POINTER(bddc_constraints), C.c_double, C.POINTER(C.c_double),
                                     C.c_int64, C.POINTER(bddc_pcg_params), C.POINTER(C.c_int64)]
    L.bddc_server_wait.argtypes = [P, C.c_int64, C.POINTER(C.c_double), C.POINTER(bddc_request_info)]
    L.bddc_server_query.argtypes = [P, C.c_int64, C.POINTER(bddc_request_info)]
    L.bddc_server_release.argtypes = [P, C.c_int64]
    L.bddc_server_destroy.argtypes = [P]
    for s in SYMBOLS:
        if s in _VOID:
            getattr(L, s).restype = None
        elif s != "bddc_last_error":
            getattr(L, s).restype = C.c_int
    _lib = L
    return L


def _ptr(a, ctype):
    return a.ctypes.data_as(C.POINTER(ctype))


# thin same-name wrappers --------------------------------------------------

def bddc_create(opt):
    h = C.c_void_p()
    _check(None, load().bddc_create(C.byref(opt), C.byref(h)))
    return h


def bddc_setup(h, mesh, part, cons):
    _check(h, load().bddc_setup(h, C.byref(mesh), C.byref(part), C.byref(cons)))


def bddc_adapt(h, tau):
    info = bddc_adapt_info()
    _check(h, load().bddc_adapt(h, float(tau), C.byref(info)))
    return info


def bddc_adapt_count(h, rows_per_face):
    info = bddc_adapt_info()
    _check(h, load().bddc_adapt_count(h, int(rows_per_face), C.byref(info)))
    return info


def bddc_factor(h):
    _check(h, load().bddc_factor(h))


def bddc_apply(h, nrhs, r_ptr, ldr, z_ptr, ldz):
    _check(h, load().bddc_apply(h, nrhs, r_ptr, ldr, z_ptr, ldz))


def bddc_apply_noalloc(h, nrhs, r_ptr, ldr, z_ptr, ldz):
    _check(h, load().bddc_apply_noalloc(h, nrhs, r_ptr, ldr, z_ptr, ldz))


def bddc_pcg_solve(h, nrhs, f_ptr, ldf, u_ptr, ldu, params, infos):
    return load().bddc_pcg_solve(h, nrhs, f_ptr, ldf, u_ptr, ldu, C.byref(params), infos)


def bddc_get_info(h):
    info = bddc_info()
    _check(h, load().bddc_get_info(h, C.byref(info)))
    return info


def bddc_last_error(h):
    return load().bddc_last_error(h).decode()


def bddc_destroy(h):
    load().bddc_destroy(h)


def _check(h, code):
    if code != 0:
        msg = bddc_last_error(h) if h is not None else ""
        raise BddcError(code, msg)


def _marshal(prob, mode, augment_corners=True, qr_drop_tol=1e-10, adaptive_edges=False):
    """ctypes structures for a meshgen-style problem, and the arrays they point to."""
    xyz = np.ascontiguousarray(prob.xyz, dtype=np.float64)
    hex8 = np.ascontiguousarray(prob.hex8, dtype=np.int64)
    coef = np.ascontiguousarray(prob.coef, dtype=np.float64)
    dirichlet = np.ascontiguousarray(prob.dirichlet, dtype=np.uint8)
    elem_sub = np.ascontiguousarray(prob.elem_sub, dtype=np.int32)
    mesh = bddc_mesh(int(prob.kind), xyz.shape[0], _ptr(xyz, C.c_double), hex8.shape[0],
                     _ptr(hex8, C.c_int64), _ptr(coef, C.c_double), float(prob.nu),
                     _ptr(dirichlet, C.c_uint8))
    part = bddc_partition(int(prob.n_sub), _ptr(elem_sub, C.c_int32))
    cons = bddc_constraints(MODES[mode] if isinstance(mode, str) else int(mode),
                            1 if augment_corners else 0, float(qr_drop_tol),
                            1 if adaptive_edges else 0)
    return mesh, part, cons, (xyz, hex8, coef, dirichlet, elem_sub)


def bddc_server_create(opt):
    h = C.c_void_p()
    _check(None, load().bddc_server_create(C.byref(opt), C.byref(h)))
    return h


def bddc_server_submit(h, mesh, part, cons, tau, f, params):
    f = np.ascontiguousarray(f, dtype=np.float64)
    rid = C.c_int64()
    _check(None, load().bddc_server_submit(h, C.byref(mesh), C.byref(part), C.byref(cons),
                                           float(tau), _ptr(f, C.c_double), f.shape[0],
                                           C.byref(params), C.byref(rid)))
    return rid.value


def bddc_server_wait(h, rid, n_glob):
    u = np.empty(n_glob, dtype=np.float64)
    info = bddc_request_info()
    _check(None, load().bddc_server_wait(h, rid, _ptr(u, C.c_double), C.byref(info)))
    return u, info


def bddc_server_query(h, rid):
    info = bddc_request_info()
    _check(None, load().bddc_server_query(h, rid, C.byref(info)))
    return info


def bddc_server_release(h, rid):
    _check(None, load().bddc_server_release(h, rid))


def bddc_server_destroy(h):
    load().bddc_server_destroy(h)


class Server:
    """Request server on one device (bddc_server_*): submit() queues a full
    setup -> adapt -> factor -> PCG solve of one problem and returns its id;
    wait() blocks for its solution (a host array) and record.  Inputs and
    results are host arrays; device memory is the server's own."""

    def __init__(self, device: int = 0, factor_precision: int = 64, max_active: int = 4,
                 hbm_budget_bytes: float = 0.0, resident_bytes: float = 0.0):
        self.h = bddc_server_create(bddc_server_options(device, factor_precision, max_active,
                                                        float(hbm_budget_bytes),
                                                        float(resident_bytes)))
        self._n = {}

    def submit(self, prob, tau=0.0, mode="ce", rtol=1e-8, maxit=1000, f=None):
        """Queues prob with load f (default prob.f)."""
        mesh, part, cons, _arrays = _marshal(prob, mode)
        f = prob.f if f is None else np.ascontiguousarray(f, dtype=np.float64)
        rid = bddc_server_submit(self.h, mesh, part, cons, tau, f, bddc_pcg_params(rtol, maxit))
        self._n[rid] = int(np.asarray(f).shape[0])
        return rid

    def wait(self, rid):
        return bddc_server_wait(self.h, rid, self._n[rid])

    def query(self, rid):
        return bddc_server_query(self.h, rid)

    def release(self, rid):
        bddc_server_release(self.h, rid)
        self._n.pop(rid, None)

    def close(self):
        if self.h is not None:
            bddc_server_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class BDDC:
    """One library context on ``device`` using torch's current stream.
    ``device < 0`` gives a host-only context (setup analysis, no GPU)."""

    def __init__(self, device: int = 0, stream=None, torch_allocator: bool = True,
                 verbose: bool = False, factor_precision: int = 64, autotune: bool = False,
                 per_substructure_launches: bool = False, chol_launch: int = 0):
        if device < 0:
            self.torch = None
            self.device = device
            opt = bddc_options()
            opt.device = device
            self._keep = []
            self.h = bddc_create(opt)
            self.n_glob = None
            _live.add(self)
            return
        import torch
        self.torch = torch
        self.device = device
        dev = torch.device("cuda", device)
        if stream is None:
            stream = torch.cuda.current_stream(dev)
        self.stream = stream
        opt = bddc_options()
        opt.device = device
        opt.hip_stream = C.c_void_p(stream.cuda_stream)
        opt.factor_precision = int(factor_precision)
        opt.verbose = 1 if verbose else 0
        opt.autotune = 1 if autotune else 0
        opt.per_substructure_launches = 1 if per_substructure_launches else 0
        opt.chol_launch = int(chol_launch)
        self._keep = []
        if torch_allocator:
            def _alloc(n, user):
                return torch.cuda.caching_allocator_alloc(int(n), device, stream)

            def _free(p, user):
                try:
                    torch.cuda.caching_allocator_delete(int(p))
                except Exception:
                    pass  # interpreter teardown: torch already gone
            fa, ff = ALLOC_FN(_alloc), FREE_FN(_free)
            self._keep += [fa, ff]
            opt.alloc, opt.free = fa, ff
        self.h = bddc_create(opt)
        self.n_glob = None
        _live.add(self)

    def close(self):
        if self.h is not None:
            bddc_destroy(self.h)
            self.h = None
        _live.discard(self)

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def setup(self, prob, mode="ce", augment_corners=True, qr_drop_tol=1e-10,
              adaptive_edges=False):
        mesh, part, cons, self._arrays = _marshal(prob, mode, augment_corners, qr_drop_tol,
                                                  adaptive_edges)
        bddc_setup(self.h, mesh, part, cons)
        self.n_glob = self.info().n_glob

    def adapt(self, tau):
        return bddc_adapt(self.h, tau)

    def adapt_count(self, rows_per_face):
        return bddc_adapt_count(self.h, rows_per_face)

    def factor(self):
        bddc_factor(self.h)

    def info(self):
        return bddc_get_info(self.h)

    def _dev(self, x):
        """Column-major device copy: returns (storage of shape (nrhs, n), n)."""
        t = self.torch
        if not isinstance(x, t.Tensor):
            x = t.as_tensor(np.asarray(x, dtype=np.float64))
        x = x.to(device=f"cuda:{self.device}", dtype=t.float64)
        if x.dim() == 1:
            x = x.unsqueeze(1)
        return x.t().contiguous(), x.shape[0]

    def apply(self, r):
        """z = M r for r of shape (n_glob,) or (n_glob, nrhs); returns (n_glob, nrhs)."""
        rt, n = self._dev(r)
        zt = self.torch.empty_like(rt)
        bddc_apply(self.h, rt.shape[0], C.c_void_p(rt.data_ptr()), n, C.c_void_p(zt.data_ptr()), n)
        return zt.t()

    def apply_noalloc(self, r, z):
        """bddc_apply_noalloc: z = M r into the caller's device tensor z, both
        (n_glob, nrhs) column-major views as returned by apply() (or 1-D);
        enqueued on the context's stream, nothing allocated by the library."""
        nr = 1 if r.dim() == 1 else r.shape[1]
        for t in (r, z):
            if not t.is_cuda or t.dtype != self.torch.float64 or t.shape[0] != self.n_glob:
                raise ValueError("r, z: float64 device tensors with n_glob rows")
            if t.dim() == 2 and (t.stride(0) != 1 or t.shape[1] != nr):
                raise ValueError("r, z: column-major (n_glob, nrhs) views of one shape")
        ldr = self.n_glob if nr == 1 else r.stride(1)
        ldz = self.n_glob if nr == 1 else z.stride(1)
        bddc_apply_noalloc(self.h, nr, C.c_void_p(r.data_ptr()), ldr, C.c_void_p(z.data_ptr()), ldz)
        return z

    def pcg_solve(self, f, rtol=1e-8, maxit=1000, raise_on_fail=True):
        ft, n = self._dev(f)
        ut = self.torch.empty_like(ft)
        nr = ft.shape[0]
        infos = (bddc_pcg_info * nr)()
        prm = bddc_pcg_params(float(rtol), int(maxit))
        code = bddc_pcg_solve(self.h, nr, C.c_void_p(ft.data_ptr()), n,
                              C.c_void_p(ut.data_ptr()), n, prm, infos)
        if code != 0 and (raise_on_fail or code != 6):
            raise BddcError(code, bddc_last_error(self.h))
        return ut.t(), [infos[i] for i in range(nr)]

    def face_rows(self, f):
        L = load()
        rows, nd = C.c_int64(), C.c_int64()
        subs = (C.c_int32 * 2)()
        _check(self.h, L.bddc_get_face_rows(self.h, f, 0, None, None, C.byref(rows), C.byref(nd), subs))
        out = np.zeros((rows.value, nd.value))
        dofs = np.zeros(nd.value, dtype=np.int64)
        _check(self.h, L.bddc_get_face_rows(self.h, f, rows.value, _ptr(out, C.c_double),
                                            _ptr(dofs, C.c_int64), C.byref(rows), C.byref(nd), subs))
        return out, dofs, (subs[0], subs[1])

    def edge_rows(self, e):
        L = load()
        rows, nd = C.c_int64(), C.c_int64()
        _check(self.h, L.bddc_get_edge_rows(self.h, e, 0, None, None, C.byref(rows), C.byref(nd)))
        out = np.zeros((rows.value, nd.value))
        dofs = np.zeros(nd.value, dtype=np.int64)
        _check(self.h, L.bddc_get_edge_rows(self.h, e, rows.value, _ptr(out, C.c_double),
                                            _ptr(dofs, C.c_int64), C.byref(rows), C.byref(nd)))
        return out, dofs

    def pcg_history(self):
        L = load()
        cnt = C.c_int64()
        _check(self.h, L.bddc_pcg_history(self.h, 0, None, C.byref(cnt)))
        out = np.zeros(cnt.value)
        _check(self.h, L.bddc_pcg_history(self.h, cnt.value, _ptr(out, C.c_double), C.byref(cnt)))
        return out

    def substructure(self, s):
        """(gdof, n_interior, scipy CSR matrix, interface weights) of substructure s."""
        import scipy.sparse as sp
        L = load()
        n, ni, nnz = C.c_int64(), C.c_int64(), C.c_int64()
        _check(self.h, L.bddc_get_substructure(self.h, s, C.byref(n), C.byref(ni), C.byref(nnz),
                                               None, None, None, None, None))
        gd = np.zeros(n.value, dtype=np.int64)
        rp = np.zeros(n.value + 1, dtype=np.int64)
        col = np.zeros(nnz.value, dtype=np.int32)
        val = np.zeros(nnz.value)
        w = np.zeros(n.value - ni.value)
        _check(self.h, L.bddc_get_substructure(self.h, s, C.byref(n), C.byref(ni), C.byref(nnz),
                                               _ptr(gd, C.c_int64), _ptr(rp, C.c_int64),
                                               _ptr(col, C.c_int32), _ptr(val, C.c_double),
                                               _ptr(w, C.c_double)))
        return gd, ni.value, sp.csr_matrix((val, col, rp), shape=(n.value, n.value)), w

    def set_timing(self, mode=1):
        """0: off; 1 (or True): phase categories; 2: every kernel launch."""
        _check(self.h, load().bddc_set_timing(self.h, int(mode)))

    def timing(self):
        """{name: dict(ms, launches, bytes, flops)} summed since set_timing."""
        L = load()
        cnt = C.c_int()
        _check(self.h, L.bddc_get_timing(self.h, 0, None, C.byref(cnt)))
        arr = (bddc_kernel_stat * max(cnt.value, 1))()
        _check(self.h, L.bddc_get_timing(self.h, cnt.value, arr, C.byref(cnt)))
        return {arr[i].name.decode(): dict(ms=arr[i].ms, launches=arr[i].launches,
                                           bytes=arr[i].bytes, flops=arr[i].flops)
                for i in range(cnt.value)}

    def face_eigs(self, f):
        L = load()
        cnt = C.c_int64()
        _check(self.h, L.bddc_get_face_eigs(self.h, f, 0, None, C.byref(cnt)))
        out = np.zeros(cnt.value)
        _check(self.h, L.bddc_get_face_eigs(self.h, f, cnt.value, _ptr(out, C.c_double), C.byref(cnt)))
        return out
