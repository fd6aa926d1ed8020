"""Python binding of the MI355X matrix-free isogeometric Karhunen-Loeve library.

The functions mirror the C ABI of include/ka.h one to one (same names,
argument marshalling only): every step of the computation runs in the HIP
library `libka.so` built from csrc/.  PyTorch is used for device memory and
streams; device arrays are passed as torch CUDA tensors.  Importing this
module fails loudly if the library has not been built.
"""
import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libka.so")

KA_OK = 0
KA_ERR_ARG = -1
KA_ERR_OOM = -2
KA_ERR_HIP = -3
KA_ERR_SINGULAR = -4
KA_ERR_STATE = -5
KA_NOT_CONVERGED = 1

KA_GALERKIN_IBQ, KA_COLLOCATION, KA_GALERKIN_GAUSS = 0, 1, 2
KA_BOX, KA_QUARTER_ANNULUS, KA_NURBS = 0, 1, 2
KA_GAUSSIAN, KA_EXP_L1 = 0, 1
KA_FP32, KA_BF16X3 = 0, 1
KA_A, KA_APRIME = 0, 1
KA_ZINV, KA_LINV, KA_LTINV = 0, 1, 2

METHODS = {"galerkin": KA_GALERKIN_IBQ, "collocation": KA_COLLOCATION, "galerkin_gauss": KA_GALERKIN_GAUSS}
DOMAINS = {"cube": KA_BOX, "box": KA_BOX, "quarter_annulus": KA_QUARTER_ANNULUS, "nurbs": KA_NURBS}
KERNELS = {"gaussian": KA_GAUSSIAN, "exponential": KA_EXP_L1}
PRECISIONS = {"fp32": KA_FP32, "bf16x3": KA_BF16X3}


class ka_desc(ctypes.Structure):
    _fields_ = [("method", ctypes.c_int), ("domain", ctypes.c_int),
                ("lo", ctypes.c_double * 3), ("hi", ctypes.c_double * 3),
                ("r0", ctypes.c_double), ("r1", ctypes.c_double), ("height", ctypes.c_double),
                ("degree", ctypes.c_int * 3), ("nel", ctypes.c_int * 3),
                ("interp_cont", ctypes.c_int), ("kernel", ctypes.c_int),
                ("sigma", ctypes.c_double), ("ell", ctypes.c_double),
                ("nq", ctypes.c_int), ("precision", ctypes.c_int), ("block", ctypes.c_int),
                ("seed", ctypes.c_ulonglong),
                ("geo_degree", ctypes.c_int * 3), ("geo_nctrl", ctypes.c_int * 3),
                ("geo_knots", ctypes.POINTER(ctypes.c_double)), ("geo_ctrl", ctypes.POINTER(ctypes.c_double))]


class ka_info(ctypes.Structure):
    _fields_ = [("iterations", ctypes.c_int), ("matvecs", ctypes.c_int), ("converged", ctypes.c_int),
                ("nev_computed", ctypes.c_int), ("max_residual", ctypes.c_double),
                ("max_imag_rel", ctypes.c_double), ("seconds", ctypes.c_double),
                ("gamma_seconds", ctypes.c_double), ("pairs", ctypes.c_double),
                ("lambda_doubles", ctypes.c_int), ("floor_accepted", ctypes.c_int)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


class ka_result(ctypes.Structure):
    _fields_ = [("id", ctypes.c_int64), ("tag", ctypes.c_uint64), ("status", ctypes.c_int), ("info", ka_info),
                ("arrival_s", ctypes.c_double), ("admit_s", ctypes.c_double), ("done_s", ctypes.c_double)]


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"HIP library not built: {LIB_PATH} is missing (run __graft_entry__.build())")
    # One HIP runtime per process: torch ships its own libamdhip64 (same soname
    # as the system one the library links).  Loading torch first makes the
    # library bind to that copy; loading the library first would map a second
    # runtime beside torch's, and streams or pointers from one are invalid in
    # the other.
    import torch  # noqa: F401
    lib = ctypes.CDLL(LIB_PATH)
    vp, i64, dp, fp = ctypes.c_void_p, ctypes.c_int64, ctypes.POINTER(ctypes.c_double), ctypes.c_void_p
    sig = {
        "ka_setup": ([ctypes.POINTER(ka_desc), vp, ctypes.POINTER(vp)], ctypes.c_int),
        "ka_size": ([vp, ctypes.POINTER(i64), ctypes.POINTER(i64), ctypes.POINTER(i64),
                     ctypes.POINTER(ctypes.c_size_t)], ctypes.c_int),
        "ka_footprint": ([ctypes.POINTER(ka_desc), ctypes.POINTER(ctypes.c_size_t)], ctypes.c_int),
        "ka_desc_size": ([ctypes.POINTER(ka_desc), ctypes.POINTER(i64), ctypes.POINTER(i64), ctypes.POINTER(i64)],
                         ctypes.c_int),
        "ka_apply_A": ([vp, ctypes.c_int, vp, i64, vp, i64, ctypes.c_int, vp], ctypes.c_int),
        "ka_solve_Z": ([vp, ctypes.c_int, vp, i64, ctypes.c_int, vp], ctypes.c_int),
        "ka_eigs": ([vp, ctypes.c_int, ctypes.c_double, ctypes.c_int, dp, i64, vp, ctypes.POINTER(ka_info)],
                    ctypes.c_int),
        "ka_gamma_apply": ([ctypes.c_int, ctypes.c_double, ctypes.c_double, fp, i64, fp, i64, fp, ctypes.c_int,
                            fp, ctypes.c_int, vp, ctypes.c_size_t, vp], ctypes.c_int),
        "ka_gamma_workspace": ([i64, i64, ctypes.c_int, ctypes.c_int], ctypes.c_size_t),
        "ka_gamma_apply_static": ([ctypes.c_int, ctypes.c_double, ctypes.c_double, fp, i64, fp, i64, fp,
                                   ctypes.c_int, fp, ctypes.c_int, vp], ctypes.c_int),
        "ka_gamma_static_capacity": ([], ctypes.c_size_t),
        "ka_profile_enable": ([vp, ctypes.c_int], ctypes.c_int),
        "ka_profile_read": ([vp, ctypes.POINTER(ctypes.c_int), dp, dp], ctypes.c_int),
        "ka_profile_reset": ([vp], ctypes.c_int),
        "ka_kl_sample": ([vp, ctypes.c_int, dp, vp, i64, ctypes.POINTER(ctypes.c_int), dp, ctypes.c_int, vp, i64,
                          ctypes.c_double, vp, i64, vp], ctypes.c_int),
        "ka_destroy": ([vp], None),
        "ka_server_create": ([ctypes.c_size_t, ctypes.c_int, ctypes.POINTER(vp)], ctypes.c_int),
        "ka_server_submit": ([vp, ctypes.POINTER(ka_desc), ctypes.c_int, ctypes.c_double, ctypes.c_int,
                              ctypes.c_double, ctypes.c_uint64, dp, i64, ctypes.POINTER(i64)], ctypes.c_int),
        "ka_server_run": ([vp, ctypes.c_double], ctypes.c_int),
        "ka_server_poll": ([vp, ctypes.POINTER(ka_result), ctypes.c_int, ctypes.POINTER(ctypes.c_int)], ctypes.c_int),
        "ka_server_stats": ([vp, ctypes.POINTER(ctypes.c_int), dp, ctypes.POINTER(ctypes.c_int),
                             ctypes.POINTER(ctypes.c_size_t)], ctypes.c_int),
        "ka_server_destroy": ([vp], None),
        "ka_request_bytes": ([ctypes.POINTER(ka_desc), ctypes.c_int, ctypes.POINTER(ctypes.c_size_t)], ctypes.c_int),
        "ka_last_error": ([], ctypes.c_char_p),
    }
    for name, (args, res) in sig.items():
        f = getattr(lib, name)
        f.argtypes = args
        f.restype = res
    return lib


_lib = _load()
EXPORTED = ("ka_setup", "ka_size", "ka_footprint", "ka_apply_A", "ka_solve_Z", "ka_eigs", "ka_gamma_apply",
            "ka_gamma_workspace", "ka_profile_enable", "ka_profile_read", "ka_profile_reset", "ka_destroy",
            "ka_last_error", "ka_server_create", "ka_server_submit", "ka_server_run", "ka_server_poll",
            "ka_server_stats", "ka_server_destroy", "ka_request_bytes", "ka_kl_sample", "ka_desc_size",
            "ka_gamma_apply_static", "ka_gamma_static_capacity")


class KAError(RuntimeError):
    def __init__(self, code, where):
        msg = _lib.ka_last_error()
        super().__init__(f"{where} failed with code {code}: {msg.decode() if msg else ''}")
        self.code = code


def _check(rc, where):
    if rc < 0:
        raise KAError(rc, where)
    return rc


def _stream(stream):
    if stream is not None:
        return ctypes.c_void_p(stream)
    import torch
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t):
    return ctypes.c_void_p(0 if t is None else t.data_ptr())


def make_desc(method, domain, p, nel, kernel, ell, sigma=1.0, block=16, precision="fp32", interp_mult=None,
              interp_cont=None, nq=None, seed=0, lo=(0.0, 0.0, 0.0), hi=(1.0, 1.0, 1.0), r0=1.0, r1=2.0,
              height=1.0, nurbs=None, **_ignored):
    """ka_desc from a plain problem descriptor (see workloads.problem).

    nurbs (domain "nurbs"): dict(degree=(p1, p2, p3), knots=(t1, t2, t3),
    ctrl=array of shape (n3, n2, n1, 4) holding x, y, z, weight).  The arrays
    are kept on the returned descriptor, so they outlive the pointers in it."""
    d = ka_desc()
    d.method = METHODS[method] if isinstance(method, str) else int(method)
    d.domain = DOMAINS[domain] if isinstance(domain, str) else int(domain)
    for k in range(3):
        d.lo[k], d.hi[k] = lo[k], hi[k]
    d.r0, d.r1, d.height = r0, r1, height
    pk = p if isinstance(p, (tuple, list)) else (p, p, p)
    for k in range(3):
        d.degree[k] = int(pk[k])
        d.nel[k] = int(nel[k])
    if interp_cont is None:
        interp_cont = -1 if interp_mult is None else int(pk[0]) - int(interp_mult)
    d.interp_cont = int(interp_cont)
    d.kernel = KERNELS[kernel] if isinstance(kernel, str) else int(kernel)
    d.sigma, d.ell = float(sigma), float(ell)
    d.nq = int(nq or 0)
    d.precision = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
    d.block = int(block)
    d.seed = int(seed)
    if nurbs is not None:
        ctrl = np.ascontiguousarray(nurbs["ctrl"], dtype=np.float64)
        if ctrl.ndim != 4 or ctrl.shape[3] != 4:
            raise ValueError("nurbs ctrl must have shape (n3, n2, n1, 4)")
        knots = np.ascontiguousarray(np.concatenate([np.asarray(t, dtype=np.float64) for t in nurbs["knots"]]))
        for k in range(3):
            d.geo_degree[k] = int(nurbs["degree"][k])
            d.geo_nctrl[k] = int(ctrl.shape[2 - k])
        d.geo_knots = knots.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
        d.geo_ctrl = ctrl.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
        d._keep = (knots, ctrl)
    return d


def desc_from_problem(prob, seed=0):
    kw = dict(prob)
    return make_desc(kw.pop("method"), kw.pop("domain"), kw.pop("p"), kw.pop("nel"), kw.pop("kernel"),
                     kw.pop("ell"), seed=seed, **kw)


# ---------------------------------------------------------------- same-name API
def ka_setup(desc, stream=None):
    h = ctypes.c_void_p()
    _check(_lib.ka_setup(ctypes.byref(desc), _stream(stream), ctypes.byref(h)), "ka_setup")
    return h


def ka_size(h):
    N, Nt, Nq, nb = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64(), ctypes.c_size_t()
    _check(_lib.ka_size(h, ctypes.byref(N), ctypes.byref(Nt), ctypes.byref(Nq), ctypes.byref(nb)), "ka_size")
    return N.value, Nt.value, Nq.value, nb.value


def ka_desc_size(desc):
    """(N, Ntilde, Nquad) that ka_setup would produce for desc (host only)."""
    N, Nt, Nq = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64()
    _check(_lib.ka_desc_size(ctypes.byref(desc), ctypes.byref(N), ctypes.byref(Nt), ctypes.byref(Nq)),
           "ka_desc_size")
    return N.value, Nt.value, Nq.value


def ka_footprint(desc):
    nb = ctypes.c_size_t()
    _check(_lib.ka_footprint(ctypes.byref(desc), ctypes.byref(nb)), "ka_footprint")
    return nb.value


def ka_apply_A(h, form, X, Y, nvec=None, stream=None):
    """X, Y: column-major FP64 device blocks, i.e. torch tensors of shape
    (nvec, N) (row j is column j of the block)."""
    nvec = X.shape[0] if nvec is None else nvec
    return _check(_lib.ka_apply_A(h, form, _ptr(X), X.shape[1], _ptr(Y), Y.shape[1], nvec, _stream(stream)),
                  "ka_apply_A")


def ka_solve_Z(h, op, X, nvec=None, stream=None):
    nvec = X.shape[0] if nvec is None else nvec
    return _check(_lib.ka_solve_Z(h, op, _ptr(X), X.shape[1], nvec, _stream(stream)), "ka_solve_Z")


def ka_eigs(h, M, tol=1e-6, maxit=100, V=None, lam=None):
    """(status, lambda, info).  lambda: M values (Galerkin methods) or 2M
    (collocation: re, im interleaved), as the library reports in
    info["lambda_doubles"].  lam: optional float64 array to write into (its
    length is passed as the capacity); by default one of 2M doubles."""
    if lam is None:
        lam = np.zeros(2 * M)
    info = ka_info()
    rc = _check(_lib.ka_eigs(h, M, tol, maxit, lam.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), lam.size,
                             _ptr(V), ctypes.byref(info)), "ka_eigs")
    return rc, lam[:info.lambda_doubles], info.as_dict()


def ka_kl_sample(h, lam, V, grid, xi, field, mu=0.0, stream=None):
    """K-L fields at a parametric tensor grid.  lam: M real eigenvalues (numpy);
    V: FP64 CUDA tensor (M, N) (row i = coefficient column i); grid: three 1-D
    arrays of parametric coordinates; xi: FP64 CUDA tensor (S, M) (row s =
    draws of sample s); field: FP64 CUDA tensor (S, P) receiving the fields
    (row s = sample s over the grid points, direction 1 fastest)."""
    lam = np.ascontiguousarray(lam, dtype=np.float64)
    M = len(lam)
    g = [np.ascontiguousarray(x, dtype=np.float64) for x in grid]
    npts = (ctypes.c_int * 3)(*[len(x) for x in g])
    gcat = np.ascontiguousarray(np.concatenate(g))
    P = int(np.prod([len(x) for x in g]))
    S = xi.shape[0]
    if V.shape[0] < M or xi.shape[1] < M or field.shape[0] != S or field.shape[1] < P:
        raise ValueError("shapes: V (M, N), xi (S, M), field (S, P)")
    return _check(_lib.ka_kl_sample(h, M, lam.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), _ptr(V), V.shape[1],
                                    npts, gcat.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), S, _ptr(xi),
                                    xi.shape[1], float(mu), _ptr(field), field.shape[1], _stream(stream)),
                  "ka_kl_sample")


def ka_gamma_workspace(nr, nc, b, precision=KA_FP32):
    return _lib.ka_gamma_workspace(nr, nc, b, precision)


def ka_gamma_apply(kernel, sigma, ell, xr, xc, Y, Z, precision=KA_FP32, work=None, stream=None):
    """xr (nr, 3), xc (nc, 3), Y (nc, b), Z (nr, b): FP32 CUDA tensors."""
    nbytes = 0 if work is None else work.numel() * work.element_size()
    return _check(_lib.ka_gamma_apply(kernel, sigma, ell, _ptr(xr), xr.shape[0], _ptr(xc), xc.shape[0], _ptr(Y),
                                      Y.shape[1], _ptr(Z), precision, _ptr(work), nbytes, _stream(stream)),
                  "ka_gamma_apply")


def ka_gamma_apply_static(kernel, sigma, ell, xr, xc, Y, Z, precision=KA_FP32, stream=None):
    """As ka_gamma_apply, with the library's static scratch (no allocation)."""
    return _check(_lib.ka_gamma_apply_static(kernel, sigma, ell, _ptr(xr), xr.shape[0], _ptr(xc), xc.shape[0],
                                             _ptr(Y), Y.shape[1], _ptr(Z), precision, _stream(stream)),
                  "ka_gamma_apply_static")


def ka_gamma_static_capacity():
    return _lib.ka_gamma_static_capacity()


def ka_profile_enable(h, on=True):
    return _check(_lib.ka_profile_enable(h, 1 if on else 0), "ka_profile_enable")


def ka_profile_read(h):
    n, ms, pairs = ctypes.c_int(), ctypes.c_double(), ctypes.c_double()
    _check(_lib.ka_profile_read(h, ctypes.byref(n), ctypes.byref(ms), ctypes.byref(pairs)), "ka_profile_read")
    return n.value, ms.value, pairs.value


def ka_profile_reset(h):
    return _check(_lib.ka_profile_reset(h), "ka_profile_reset")


def ka_destroy(h):
    if h:
        _lib.ka_destroy(h)


def ka_last_error():
    m = _lib.ka_last_error()
    return m.decode() if m else ""


def ka_request_bytes(desc, M):
    nb = ctypes.c_size_t()
    _check(_lib.ka_request_bytes(ctypes.byref(desc), M, ctypes.byref(nb)), "ka_request_bytes")
    return nb.value


def ka_server_create(hbm_budget, max_slots):
    h = ctypes.c_void_p()
    _check(_lib.ka_server_create(int(hbm_budget), int(max_slots), ctypes.byref(h)), "ka_server_create")
    return h


def ka_server_submit(srv, desc, M, lam, tol=1e-5, maxit=60, arrival_s=0.0, tag=0):
    """lam: caller-owned float64 numpy array of at least M (Galerkin) or 2M
    (collocation) entries; it must stay alive until the request completes."""
    rid = ctypes.c_int64()
    _check(_lib.ka_server_submit(srv, ctypes.byref(desc), M, tol, maxit, arrival_s, tag,
                                 lam.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), lam.size, ctypes.byref(rid)),
           "ka_server_submit")
    return rid.value


def ka_server_run(srv, timeout_s=0.0):
    return _check(_lib.ka_server_run(srv, timeout_s), "ka_server_run")


def ka_server_poll(srv, max_results=4096):
    buf = (ka_result * max_results)()
    n = ctypes.c_int()
    _check(_lib.ka_server_poll(srv, buf, max_results, ctypes.byref(n)), "ka_server_poll")
    out = []
    for i in range(n.value):
        r = buf[i]
        out.append(dict(id=r.id, tag=r.tag, status=r.status, info=r.info.as_dict(), arrival_s=r.arrival_s,
                        admit_s=r.admit_s, done_s=r.done_s))
    return out


def ka_server_stats(srv):
    b, mi, ma, used = ctypes.c_int(), ctypes.c_double(), ctypes.c_int(), ctypes.c_size_t()
    _check(_lib.ka_server_stats(srv, ctypes.byref(b), ctypes.byref(mi), ctypes.byref(ma), ctypes.byref(used)),
           "ka_server_stats")
    return dict(batches=b.value, mean_items=mi.value, max_active=ma.value, bytes_in_use=used.value)


def ka_server_destroy(srv):
    if srv:
        _lib.ka_server_destroy(srv)


class Problem:
    """Owning wrapper around a ka_problem handle."""

    def __init__(self, desc, stream=None):
        self.desc = desc
        self.h = ka_setup(desc, stream)
        self.N, self.Ntilde, self.Nquad, self.device_bytes = ka_size(self.h)

    def close(self):
        if self.h:
            ka_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
