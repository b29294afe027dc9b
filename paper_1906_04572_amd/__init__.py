"""Python binding of libcorutv (CoR-UTV and ALM-CoRUTV robust PCA on MI355X).

Argument marshalling only: torch supplies device memory and streams, every
step of the computation runs in the HIP library.  The library is loaded from
this package directory; importing fails loudly if it has not been built
(``python -m paper_1906_04572_amd._build`` or ``__graft_entry__.build()``).
"""
import ctypes
import os

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libcorutv.so")

OK, PENDING = 0, 1
E_INVAL, E_NOMEM, E_BUSY, E_NUMERIC, E_DEVICE, E_NOTFOUND = -1, -2, -3, -4, -5, -6
FLAG_CORE_FROM_RZ = 1  # core D = R_Z^T (2q + 2 passes)
FLAG_A_HOST = 2  # A in host memory, streamed through the device in panels
CORE = {"pass": 0, "rz": FLAG_CORE_FROM_RZ}
F64, F32 = 0, 1
COL_MAJOR, ROW_MAJOR = 0, 1
PREC = {"f64": 0, "f32": 1, "bf16": 2, "bf16x3": 3}
TRI = {"auto": 0, "upper": 1, "lower": 2}
TRI_NAME = {1: "upper", 2: "lower"}


class CorutvError(RuntimeError):
    def __init__(self, code, what=""):
        self.code = code
        super().__init__("%s (%d)%s" % (strerror(code), code, (": " + what) if what else ""))


class Mat(ctypes.Structure):
    _fields_ = [("ptr", ctypes.c_void_p), ("rows", ctypes.c_int64), ("cols", ctypes.c_int64),
                ("ld", ctypes.c_int64), ("dtype", ctypes.c_int32), ("layout", ctypes.c_int32)]


class Opts(ctypes.Structure):
    _fields_ = [("prec", ctypes.c_int32), ("tri", ctypes.c_int32), ("want_err", ctypes.c_int32),
                ("flags", ctypes.c_int32), ("panel_rows", ctypes.c_int32)]


class Info(ctypes.Structure):
    _fields_ = [("rel_err", ctypes.c_double), ("a_fro", ctypes.c_double), ("gpu_ms", ctypes.c_double),
                ("ell", ctypes.c_int32), ("transposed", ctypes.c_int32), ("tri", ctypes.c_int32),
                ("qr_fallbacks", ctypes.c_int32), ("passes", ctypes.c_int32),
                ("qr_one_step", ctypes.c_int32)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


class RpcaInfo(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int32), ("final_rank", ctypes.c_int32), ("zeta", ctypes.c_double),
                ("mu0", ctypes.c_double), ("mu", ctypes.c_double), ("gpu_ms", ctypes.c_double),
                ("step_ms", ctypes.c_double)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


class PassStats(ctypes.Structure):
    _fields_ = [("passes", ctypes.c_int64), ("total_ms", ctypes.c_double), ("min_ms", ctypes.c_double),
                ("max_ms", ctypes.c_double)]


class Config(ctypes.Structure):
    _fields_ = [("device", ctypes.c_int32), ("n_streams", ctypes.c_int32),
                ("streams", ctypes.POINTER(ctypes.c_void_p)), ("workspace", ctypes.c_void_p),
                ("workspace_bytes", ctypes.c_uint64), ("max_queue", ctypes.c_int32),
                ("flags", ctypes.c_uint32)]


class Request(ctypes.Structure):
    _fields_ = [("A", Mat), ("U", Mat), ("V", Mat), ("T", ctypes.c_void_p), ("ldt", ctypes.c_int64),
                ("piv", ctypes.c_void_p), ("k", ctypes.c_int32), ("p", ctypes.c_int32),
                ("q", ctypes.c_int32), ("priority", ctypes.c_int32), ("seed", ctypes.c_uint64),
                ("opts", Opts)]


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError("libcorutv.so is not built (%s); run __graft_entry__.build()" % LIB_PATH)
    lib = ctypes.CDLL(LIB_PATH)
    P, I32, I64, U64, D = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_uint64, ctypes.c_double
    MP = ctypes.POINTER(Mat)
    sig = {
        "corutv_create": (ctypes.c_int, [ctypes.POINTER(P), ctypes.POINTER(Config)]),
        "corutv_destroy": (ctypes.c_int, [P]),
        "corutv_workspace_bytes": (U64, [I64, I64, I32, I32, I32, I32]),
        "corutv_workspace_bytes_host": (U64, [I64, I64, I32, I32, I32, I32, I32, I32]),
        "corutv_decompose": (ctypes.c_int, [P, MP, I32, I32, I32, U64, ctypes.POINTER(Opts), MP, P, I64,
                                            MP, P, ctypes.POINTER(Info)]),
        "corutv_decompose_noalloc": (ctypes.c_int, [P, MP, I32, I32, I32, U64, ctypes.POINTER(Opts), MP, P,
                                                    I64, MP, P, ctypes.POINTER(Info)]),
        "corutv_rpca": (ctypes.c_int, [P, MP, D, I32, I32, I32, I32, D, U64, ctypes.POINTER(Opts), MP, MP,
                                       ctypes.POINTER(RpcaInfo)]),
        "corutv_submit": (ctypes.c_int, [P, ctypes.POINTER(Request), ctypes.POINTER(U64)]),
        "corutv_poll": (ctypes.c_int, [P, U64, ctypes.POINTER(Info)]),
        "corutv_wait": (ctypes.c_int, [P, U64, ctypes.POINTER(Info)]),
        "corutv_cancel": (ctypes.c_int, [P, U64]),
        "corutv_strerror": (ctypes.c_char_p, [ctypes.c_int]),
        "corutv_omega": (ctypes.c_int, [P, I64, I32, U64, ctypes.c_uint32, I32, P, I64]),
        "corutv_sketch": (ctypes.c_int, [P, MP, I32, I32, P, I64, I32, P, I64]),
        "corutv_tsqr": (ctypes.c_int, [P, P, I64, I32, I64, P, I64, P, I64, ctypes.POINTER(I32)]),
        "corutv_qrcp": (ctypes.c_int, [P, I32, P, I64, P, P, P]),
        "corutv_rpca_workspace_bytes": (U64, [I64, I64, I32, I32, I32]),
        "corutv_rpca_ranks": (ctypes.c_int, [P, ctypes.POINTER(I32), I32, ctypes.POINTER(I32)]),
        "corutv_pass_timing": (ctypes.c_int, [P, I32, I32]),
        "corutv_get_pass_stats": (ctypes.c_int, [P, ctypes.POINTER(PassStats)]),
        "corutv_debug_inject_failure": (ctypes.c_int, [P, I32]),
    }
    for name, (res, args) in sig.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    return lib


lib = _load()


def strerror(code):
    return lib.corutv_strerror(code).decode()


def _check(rc, what=""):
    if rc != OK:
        raise CorutvError(rc, what)
    return rc


def mat(t, host=False):
    """Descriptor of a 2-D CUDA tensor (row-major contiguous or a transposed
    view of one, i.e. column-major); host=True takes a CPU tensor instead."""
    if t.dim() != 2 or t.is_cuda == host:
        raise ValueError("expected a 2-D %s tensor" % ("host" if host else "device"))
    dt = {torch.float64: F64, torch.float32: F32}.get(t.dtype)
    if dt is None:
        raise ValueError("dtype must be float64 or float32")
    r, c = t.shape
    s0, s1 = t.stride()
    if s1 == 1 and (s0 >= c or r == 1):
        return Mat(t.data_ptr(), r, c, max(s0, c), dt, ROW_MAJOR)
    if s0 == 1 and (s1 >= r or c == 1):
        return Mat(t.data_ptr(), r, c, max(s1, r), dt, COL_MAJOR)
    raise ValueError("tensor must be row- or column-major with unit inner stride")


def workspace_bytes(m, n, k, p, q, prec="f64"):
    return int(lib.corutv_workspace_bytes(m, n, k, p, q, PREC[prec]))


def workspace_bytes_host(m, n, k, p, q, prec="f64", layout="row", panel_rows=0):
    """Workspace for a host-resident A (two staging panels included)."""
    return int(lib.corutv_workspace_bytes_host(m, n, k, p, q, PREC[prec],
                                               ROW_MAJOR if layout == "row" else COL_MAJOR, panel_rows))


def rpca_workspace_bytes(m, n, k, p, q):
    return int(lib.corutv_rpca_workspace_bytes(m, n, k, p, q))


class Context:
    """A libcorutv context bound to one device, a workspace tensor and streams.

    ``streams``: list of torch.cuda.Stream; the first is the context stream,
    the others are serving slots.
    """

    def __init__(self, workspace_bytes=1 << 30, device=0, streams=None, max_queue=0):
        self.device = torch.device("cuda", device)
        # workspace_bytes = 0: no workspace (corutv_decompose_noalloc only)
        self.ws = torch.empty(int(workspace_bytes), dtype=torch.uint8, device=self.device)
        if streams is None:
            streams = [torch.cuda.current_stream(self.device)]
        self.streams = list(streams)
        arr = (ctypes.c_void_p * len(self.streams))(*[s.cuda_stream for s in self.streams])
        self._arr = arr
        cfg = Config(device, len(self.streams), ctypes.cast(arr, ctypes.POINTER(ctypes.c_void_p)),
                     self.ws.data_ptr(), self.ws.numel(), max_queue, 0)
        h = ctypes.c_void_p()
        _check(lib.corutv_create(ctypes.byref(h), ctypes.byref(cfg)), "create")
        self.h = h
        self._live = {}

    def close(self):
        if self.h:
            lib.corutv_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- decomposition ------------------------------------------------------
    def alloc_outputs(self, A, k, p, dtype=None, layout="col"):
        m, n = A.shape
        ell = k + p
        dt = dtype or A.dtype
        dev = self.device
        if layout == "col":
            U = torch.zeros((ell, m), dtype=dt, device=dev).t()
            V = torch.zeros((ell, n), dtype=dt, device=dev).t()
        else:
            U = torch.zeros((m, ell), dtype=dt, device=dev)
            V = torch.zeros((n, ell), dtype=dt, device=dev)
        T = torch.zeros((ell, ell), dtype=torch.float64, device=dev).t()  # column-major
        piv = torch.zeros(ell, dtype=torch.int32, device=dev)
        return U, T, V, piv

    def decompose(self, A, k, p, q, seed, prec="f64", tri="auto", want_err=False, out=None, core="pass",
                  panel_rows=0):
        """Returns (U, T, V, piv, info dict).  core: "pass" (D = Q1^T (A Q2)) or
        "rz" (D = R_Z^T from the QR of the second sketch, one pass fewer).
        A CPU tensor A (pinned for overlap) is streamed through the device in
        panels of panel_rows storage rows (0: the library default)."""
        U, T, V, piv = out if out is not None else self.alloc_outputs(A, k, p)
        ell = k + p
        info = Info()
        host = not A.is_cuda
        opts = Opts(PREC[prec], TRI[tri], 1 if want_err else 0, CORE[core] | (FLAG_A_HOST if host else 0),
                    panel_rows)
        mu, mv = mat(U), mat(V)
        rc = lib.corutv_decompose(self.h, ctypes.byref(mat(A, host)), k, p, q, seed, ctypes.byref(opts),
                                  ctypes.byref(mu), T.data_ptr(), ell, ctypes.byref(mv), piv.data_ptr(),
                                  ctypes.byref(info))
        _check(rc, "decompose")
        d = info.as_dict()
        d["tri"] = TRI_NAME.get(d["tri"], d["tri"])
        return U, T, V, piv, d

    def decompose_noalloc(self, A, k, p, q, seed, prec="f64", tri="auto", want_err=False, out=None,
                          core="pass"):
        """decompose() through corutv_decompose_noalloc: scratch from the
        library's fixed per-device array instead of the context workspace."""
        U, T, V, piv = out if out is not None else self.alloc_outputs(A, k, p)
        info = Info()
        opts = Opts(PREC[prec], TRI[tri], 1 if want_err else 0, CORE[core], 0)
        mu, mv = mat(U), mat(V)
        rc = lib.corutv_decompose_noalloc(self.h, ctypes.byref(mat(A)), k, p, q, seed, ctypes.byref(opts),
                                          ctypes.byref(mu), T.data_ptr(), k + p, ctypes.byref(mv),
                                          piv.data_ptr(), ctypes.byref(info))
        _check(rc, "decompose_noalloc")
        d = info.as_dict()
        d["tri"] = TRI_NAME.get(d["tri"], d["tri"])
        return U, T, V, piv, d

    def decompose_rc(self, A, k, p, q, seed, prec="f64", tri="auto", want_err=False, out=None, core="pass",
                     panel_rows=0):
        """Like decompose but returns the status code instead of raising."""
        U, T, V, piv = out if out is not None else self.alloc_outputs(A, k, p)
        info = Info()
        host = not A.is_cuda
        opts = Opts(PREC[prec], TRI[tri], 1 if want_err else 0, CORE[core] | (FLAG_A_HOST if host else 0),
                    panel_rows)
        mu, mv = mat(U), mat(V)
        return lib.corutv_decompose(self.h, ctypes.byref(mat(A, host)), k, p, q, seed, ctypes.byref(opts),
                                    ctypes.byref(mu), T.data_ptr(), k + p, ctypes.byref(mv),
                                    piv.data_ptr(), ctypes.byref(info))

    # -- single steps -------------------------------------------------------
    def omega(self, n, ell, seed, sub=0, dtype=torch.float64):
        out = torch.empty((ell, n), dtype=dtype, device=self.device)  # column-major n x ell
        _check(lib.corutv_omega(self.h, n, ell, seed, sub, F64 if dtype == torch.float64 else F32,
                                out.data_ptr(), n), "omega")
        return out.t()

    def sketch(self, A, X, trans=False, prec="f64"):
        """Y = A X (trans False) or A^T X, X column-major (rows x ell)."""
        ell = X.shape[1]
        Xc = X.t().contiguous()  # (ell, rows) row-major == column-major X
        rows_out = A.shape[1] if trans else A.shape[0]
        Y = torch.empty((ell, rows_out), dtype=X.dtype, device=self.device)
        _check(lib.corutv_sketch(self.h, ctypes.byref(mat(A)), 1 if trans else 0, PREC[prec],
                                 Xc.data_ptr(), Xc.shape[1], ell, Y.data_ptr(), rows_out), "sketch")
        return Y.t()

    def tsqr(self, X):
        rows, ell = X.shape
        Xc = X.t().contiguous()
        Q = torch.empty((ell, rows), dtype=torch.float64, device=self.device)
        R = torch.zeros((ell, ell), dtype=torch.float64, device=self.device)
        fb = ctypes.c_int32(0)
        _check(lib.corutv_tsqr(self.h, Xc.data_ptr(), rows, ell, rows, Q.data_ptr(), rows, R.data_ptr(),
                               ell, ctypes.byref(fb)), "tsqr")
        return Q.t(), R.t(), bool(fb.value)

    def qrcp(self, D):
        ell = D.shape[0]
        Dc = D.t().contiguous()
        Qt = torch.empty((ell, ell), dtype=torch.float64, device=self.device)
        R = torch.empty((ell, ell), dtype=torch.float64, device=self.device)
        piv = torch.empty(ell, dtype=torch.int32, device=self.device)
        _check(lib.corutv_qrcp(self.h, ell, Dc.data_ptr(), ell, Qt.data_ptr(), R.data_ptr(),
                               piv.data_ptr()), "qrcp")
        return Qt.t(), R.t(), piv

    # -- measurement ----------------------------------------------------------
    def pass_timing(self, enable=True, reset=True):
        _check(lib.corutv_pass_timing(self.h, 1 if enable else 0, 1 if reset else 0), "pass_timing")

    def inject_failure(self, after_checks):
        """Test hook: the n-th next launch check fails as a HIP error would."""
        _check(lib.corutv_debug_inject_failure(self.h, after_checks), "inject_failure")

    def pass_stats(self):
        st = PassStats()
        _check(lib.corutv_get_pass_stats(self.h, ctypes.byref(st)), "pass_stats")
        return {f: getattr(st, f) for f, _ in st._fields_}

    # -- robust PCA -----------------------------------------------------------
    def rpca(self, M, k, p, q, seed, lam=-1.0, max_iter=50, tol=0.0, want_L=True):
        """Returns (L or None, S, info dict).  M float32 (either layout)."""
        S = torch.zeros((M.shape[1], M.shape[0]), dtype=torch.float32, device=self.device).t()
        L = torch.zeros_like(S) if want_L else None
        info = RpcaInfo()
        opts = Opts(PREC["f32"], 0, 0, 0)
        ms = mat(S)
        ml = mat(L) if L is not None else None
        rc = lib.corutv_rpca(self.h, ctypes.byref(mat(M)), lam, k, p, q, max_iter, tol, seed,
                             ctypes.byref(opts), ctypes.byref(ml) if ml is not None else None,
                             ctypes.byref(ms), ctypes.byref(info))
        _check(rc, "rpca")
        out = info.as_dict()
        out["ranks"] = self.rpca_ranks()
        return L, S, out

    def rpca_ranks(self):
        """r_j of every iteration of the last rpca call (up to 4096)."""
        cnt = ctypes.c_int32()
        _check(lib.corutv_rpca_ranks(self.h, None, 0, ctypes.byref(cnt)), "rpca_ranks")
        buf = (ctypes.c_int32 * max(cnt.value, 1))()
        _check(lib.corutv_rpca_ranks(self.h, buf, cnt.value, None), "rpca_ranks")
        return [int(buf[i]) for i in range(cnt.value)]

    # -- serving --------------------------------------------------------------
    def submit(self, A, k, p, q, seed, prec="f64", tri="auto", want_err=False, out=None, core="pass"):
        U, T, V, piv = out if out is not None else self.alloc_outputs(A, k, p)
        req = Request(mat(A), mat(U), mat(V), T.data_ptr(), k + p, piv.data_ptr(), k, p, q, 0, seed,
                      Opts(PREC[prec], TRI[tri], 1 if want_err else 0, CORE[core]))
        t = ctypes.c_uint64(0)
        _check(lib.corutv_submit(self.h, ctypes.byref(req), ctypes.byref(t)), "submit")
        self._live[t.value] = (A, U, T, V, piv)
        return t.value

    def poll(self, ticket):
        info = Info()
        rc = lib.corutv_poll(self.h, ticket, ctypes.byref(info))
        if rc == PENDING:
            return None
        bufs = self._live.pop(ticket, None)
        _check(rc, "poll")
        _, U, T, V, piv = bufs
        return U, T, V, piv, info.as_dict()

    def wait(self, ticket):
        info = Info()
        rc = lib.corutv_wait(self.h, ticket, ctypes.byref(info))
        bufs = self._live.pop(ticket, None)
        _check(rc, "wait")
        _, U, T, V, piv = bufs
        return U, T, V, piv, info.as_dict()
