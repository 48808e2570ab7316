"""ctypes binding of the C ABI in include/sos.h (argument marshalling only).

Every function here converts Python/numpy arguments into the plain pointers and
sizes of the C ABI and calls libsos.so; all solver work runs in the library's
gfx950 kernels.  If the library has not been built, importing this module fails
loudly: there is no CPU fallback.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import List, Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libsos.so")

SOS_OK, SOS_E_INVAL, SOS_E_ASYM, SOS_E_NOMEM, SOS_E_HIP, SOS_E_STATE = 0, -1, -2, -3, -4, -5
SOS_UNSOLVED, SOS_SOLVED, SOS_PRIMAL_INFEASIBLE, SOS_DUAL_INFEASIBLE, SOS_MAX_ITERS = 0, 1, 2, 3, 4
SOS_FP64, SOS_FP32_MIXED = 0, 1
SOS_PART_PAPER, SOS_PART_COLUMNS = 0, 1
STATUS_NAMES = {0: "unsolved", 1: "solved", 2: "primal_infeasible", 3: "dual_infeasible", 4: "max_iters"}

EXPORTED = ["sos_default_settings", "sos_setup", "sos_step", "sos_step_static", "sos_solve", "sos_warm_start",
            "sos_get_solution", "sos_get_iterate", "sos_set_iterate", "sos_psd_factor", "sos_get_eig_cache",
            "sos_last_error", "sos_free",
            "sos_batch_setup", "sos_batch_solve", "sos_batch_reset", "sos_batch_last_ms", "sos_batch_last_error",
            "sos_batch_phase_ms", "sos_batch_free", "sos_layout_size", "sos_batch_warm_start",
            "sos_batch_export_solutions", "sos_mlp_create", "sos_mlp_num_params", "sos_mlp_set_params",
            "sos_mlp_get_params", "sos_mlp_set_output_affine", "sos_mlp_forward", "sos_mlp_gradient",
            "sos_mlp_train_step", "sos_mlp_train_step_rows", "sos_mlp_free"]


class SosError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"sos error {code}: {msg}")
        self.code = code


class sos_csc(C.Structure):
    _fields_ = [("m", C.c_int32), ("n", C.c_int32), ("colptr", C.POINTER(C.c_int64)),
                ("rowind", C.POINTER(C.c_int32)), ("val", C.POINTER(C.c_double))]


class sos_cone(C.Structure):
    _fields_ = [("n_free", C.c_int32), ("n_psd", C.c_int32), ("N", C.POINTER(C.c_int32))]


class sos_settings(C.Structure):
    _fields_ = [("tol", C.c_double), ("max_iters", C.c_int32), ("check_every", C.c_int32),
                ("alpha", C.c_double), ("precision", C.c_int32), ("polish_iters", C.c_int32),
                ("partition", C.c_int32), ("block_threads", C.c_int32), ("eig_form", C.c_int32),
                ("warm_budget", C.c_int32), ("scale_iters", C.c_int32)]


class sos_info(C.Structure):
    _fields_ = [("status", C.c_int32), ("iters", C.c_int32), ("k_lowrank", C.c_int32),
                ("polish_iters", C.c_int32), ("pobj", C.c_double), ("dobj", C.c_double),
                ("res_pri", C.c_double), ("res_dual", C.c_double), ("gap", C.c_double),
                ("tau", C.c_double), ("kappa", C.c_double), ("setup_ms", C.c_double),
                ("solve_ms", C.c_double), ("eig_sweeps", C.c_double), ("affine_ms", C.c_double),
                ("eig_ms", C.c_double), ("resid_ms", C.c_double), ("warm_iters", C.c_int32),
                ("start_ms", C.c_double), ("end_ms", C.c_double)]

    def as_dict(self) -> dict:
        d = {f: getattr(self, f) for f, _ in self._fields_}
        d["status_name"] = STATUS_NAMES.get(self.status, str(self.status))
        return d


_lib = None


def load():
    """Loads libsos.so (raises if it was not built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with __graft_entry__.build() "
                          "(the solver has no CPU fallback)")
    try:
        import torch  # noqa: F401  - one HIP runtime per process: the one torch brings
    except Exception:
        pass
    lib = C.CDLL(LIB_PATH)
    P = C.POINTER
    vp = C.c_void_p
    lib.sos_default_settings.argtypes = [P(sos_settings)]
    lib.sos_setup.argtypes = [P(sos_csc), P(C.c_double), P(C.c_double), P(sos_cone), P(sos_settings), vp, P(vp)]
    lib.sos_step.argtypes = [vp, C.c_int32, P(sos_info)]
    lib.sos_step_static.argtypes = [vp, C.c_int32, P(sos_info)]
    lib.sos_solve.argtypes = [vp, P(sos_info)]
    lib.sos_warm_start.argtypes = [vp, P(C.c_double), P(C.c_double), P(C.c_double), C.c_double, C.c_double]
    lib.sos_get_solution.argtypes = [vp, P(C.c_double), P(C.c_double), P(C.c_double)]
    lib.sos_get_iterate.argtypes = [vp, P(C.c_double), P(C.c_double)]
    lib.sos_set_iterate.argtypes = [vp, P(C.c_double), P(C.c_double)]
    lib.sos_psd_factor.argtypes = [vp, C.c_int32, C.c_int32, P(C.c_double), P(C.c_double)]
    lib.sos_get_eig_cache.argtypes = [vp, C.c_int32, C.c_int32, P(C.c_double), P(C.c_int32)]
    lib.sos_last_error.argtypes = [vp]
    lib.sos_last_error.restype = C.c_char_p
    lib.sos_free.argtypes = [vp]
    lib.sos_free.restype = None
    lib.sos_batch_setup.argtypes = [C.c_int32, P(vp), C.c_char_p, P(vp)]
    lib.sos_batch_solve.argtypes = [vp, P(sos_info)]
    lib.sos_batch_reset.argtypes = [vp]
    lib.sos_batch_last_ms.argtypes = [vp]
    lib.sos_batch_last_ms.restype = C.c_double
    lib.sos_batch_phase_ms.argtypes = [vp, C.c_int32]
    lib.sos_batch_phase_ms.restype = C.c_double
    lib.sos_batch_free.argtypes = [vp]
    lib.sos_batch_last_error.argtypes = [vp]
    lib.sos_batch_last_error.restype = C.c_char_p
    lib.sos_batch_free.restype = None
    fp = P(C.c_float)
    lib.sos_layout_size.argtypes = [vp]
    lib.sos_layout_size.restype = C.c_int64
    lib.sos_batch_warm_start.argtypes = [vp, vp, C.c_int64]
    lib.sos_batch_export_solutions.argtypes = [vp, vp, C.c_int64]
    lib.sos_mlp_create.argtypes = [C.c_int32, C.c_int32, C.c_int32, C.c_int32, vp, P(vp)]
    lib.sos_mlp_num_params.argtypes = [vp]
    lib.sos_mlp_num_params.restype = C.c_int64
    lib.sos_mlp_set_params.argtypes = [vp, fp]
    lib.sos_mlp_get_params.argtypes = [vp, fp]
    lib.sos_mlp_set_output_affine.argtypes = [vp, fp, fp]
    lib.sos_mlp_forward.argtypes = [vp, vp, C.c_int32, vp, C.c_int32]
    lib.sos_mlp_gradient.argtypes = [vp, vp, vp, C.c_int32, fp, P(C.c_double)]
    lib.sos_mlp_train_step.argtypes = [vp, vp, vp, C.c_int32, C.c_float, P(C.c_double)]
    lib.sos_mlp_train_step_rows.argtypes = [vp, vp, vp, vp, C.c_int32, C.c_float, P(C.c_double)]
    lib.sos_mlp_free.argtypes = [vp]
    lib.sos_mlp_free.restype = None
    for name in EXPORTED:
        if name not in ("sos_free", "sos_batch_free", "sos_last_error", "sos_batch_last_error", "sos_batch_last_ms",
                        "sos_batch_phase_ms",
                        "sos_layout_size", "sos_mlp_num_params", "sos_mlp_free"):
            getattr(lib, name).restype = C.c_int
    _lib = lib
    return lib


def _dptr(a: np.ndarray):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _check(rc: int, handle=None, batch=None):
    if rc != SOS_OK:
        msg = load().sos_batch_last_error(batch) if batch is not None else load().sos_last_error(handle)
        raise SosError(rc, msg.decode() if msg else "")


def current_stream():
    """hipStream_t of torch's current stream on cuda:0, or None (the NULL stream)."""
    try:
        import torch
        if torch.cuda.is_available():
            return C.c_void_p(torch.cuda.current_stream().cuda_stream)
    except Exception:
        pass
    return None


def sos_default_settings(**overrides) -> sos_settings:
    s = sos_settings()
    _check(load().sos_default_settings(C.byref(s)))
    for k, v in overrides.items():
        if not hasattr(s, k):
            raise KeyError(k)
        setattr(s, k, v)
    return s


class Work:
    """Owns one sos_work handle; the arrays it describes stay readable via the methods below."""

    def __init__(self, handle: C.c_void_p, n: int, m: int, psd_dims=()):
        self.handle = handle
        self.n, self.m = n, m
        self.psd_dims = list(psd_dims)

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass

    def free(self):
        if self.handle:
            load().sos_free(self.handle)
            self.handle = None


def sos_setup(A, b, c, n_free: int, psd_dims: Sequence[int], settings: Optional[sos_settings] = None,
              stream=None) -> Work:
    """A: scipy.sparse matrix (m x n, full column-stacked vec); b (m); c (n)."""
    import scipy.sparse as sp
    lib = load()
    A = sp.csc_matrix(A)
    A.sort_indices()
    colptr = np.ascontiguousarray(A.indptr, dtype=np.int64)
    rowind = np.ascontiguousarray(A.indices, dtype=np.int32)
    val = np.ascontiguousarray(A.data, dtype=np.float64)
    b = np.ascontiguousarray(b, dtype=np.float64)
    c = np.ascontiguousarray(c, dtype=np.float64)
    Ns = np.ascontiguousarray(psd_dims, dtype=np.int32)
    csc = sos_csc(A.shape[0], A.shape[1], colptr.ctypes.data_as(C.POINTER(C.c_int64)),
                  rowind.ctypes.data_as(C.POINTER(C.c_int32)), _dptr(val))
    cone = sos_cone(n_free, len(Ns), Ns.ctypes.data_as(C.POINTER(C.c_int32)))
    h = C.c_void_p()
    st = stream if stream is not None else current_stream()
    rc = lib.sos_setup(C.byref(csc), _dptr(b), _dptr(c), C.byref(cone),
                       C.byref(settings) if settings is not None else None, st, C.byref(h))
    _check(rc, None)
    return Work(h, A.shape[1], A.shape[0], [int(x) for x in Ns])


def setup_problem(prob, settings: Optional[sos_settings] = None, stream=None) -> Work:
    return sos_setup(prob.A, prob.b, prob.c, prob.n_free, prob.psd_dims, settings, stream)


def sos_step(w: Work, iters: int) -> dict:
    info = sos_info()
    _check(load().sos_step(w.handle, int(iters), C.byref(info)), w.handle)
    return info.as_dict()


def sos_step_static(w: Work, iters: int) -> dict:
    """sos_step with the launch scratch in the library's static device array (no allocation)."""
    info = sos_info()
    _check(load().sos_step_static(w.handle, int(iters), C.byref(info)), w.handle)
    return info.as_dict()


def sos_solve(w: Work) -> dict:
    info = sos_info()
    _check(load().sos_solve(w.handle, C.byref(info)), w.handle)
    return info.as_dict()


def sos_warm_start(w: Work, x, y, z, tau: float = 1.0, kappa: float = 0.0) -> None:
    x = np.ascontiguousarray(x, dtype=np.float64)
    y = np.ascontiguousarray(y, dtype=np.float64)
    z = np.ascontiguousarray(z, dtype=np.float64)
    if x.shape != (w.n,) or z.shape != (w.n,) or y.shape != (w.m,):
        raise ValueError("warm start has the wrong shape")
    _check(load().sos_warm_start(w.handle, _dptr(x), _dptr(y), _dptr(z), float(tau), float(kappa)), w.handle)


def sos_get_solution(w: Work):
    x, y, z = np.empty(w.n), np.empty(w.m), np.empty(w.n)
    _check(load().sos_get_solution(w.handle, _dptr(x), _dptr(y), _dptr(z)), w.handle)
    return x, y, z


def sos_get_iterate(w: Work):
    u = np.empty(w.n + w.m + 1)
    v = np.empty(w.n + w.m + 1)
    _check(load().sos_get_iterate(w.handle, _dptr(u), _dptr(v)), w.handle)
    return u, v


def sos_set_iterate(w: Work, u, v) -> None:
    u = np.ascontiguousarray(u, dtype=np.float64)
    v = np.ascontiguousarray(v, dtype=np.float64)
    if u.shape != (w.n + w.m + 1,) or v.shape != (w.n + w.m + 1,):
        raise ValueError("iterate has the wrong shape")
    _check(load().sos_set_iterate(w.handle, _dptr(u), _dptr(v)), w.handle)


def sos_psd_factor(w: Work, block: int, dual: bool = False):
    """(evals (N), evecs (N x N)) of block `block` of X = xi / tau, or of Z = z / tau if dual."""
    N = int(w.psd_dims[block]) if 0 <= block < len(w.psd_dims) else 1   # a bad index: the library says so
    lam = np.empty(N)
    vec = np.empty(N * N)
    _check(load().sos_psd_factor(w.handle, int(block), int(bool(dual)), _dptr(lam), _dptr(vec)), w.handle)
    return lam, vec.reshape(N, N, order="F")


def sos_get_eig_cache(w: Work, block: int, precision: int = SOS_FP64):
    """(V (N x N, columns = the cached eigenvectors of block `block`), valid) from the warm-start
    cache of the given precision."""
    N = int(w.psd_dims[block]) if 0 <= block < len(w.psd_dims) else 1
    vec = np.empty(N * N)
    valid = C.c_int32(0)
    _check(load().sos_get_eig_cache(w.handle, int(block), int(precision), _dptr(vec), C.byref(valid)), w.handle)
    return vec.reshape(N, N, order="F"), bool(valid.value)


def sos_free(w: Work) -> None:
    w.free()


class Batch:
    def __init__(self, handle, works: List[Work]):
        self.handle = handle
        self.works = works      # keeps the handles alive

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass

    def free(self):
        if self.handle:
            load().sos_batch_free(self.handle)
            self.handle = None


def sos_batch_setup(works: Sequence[Work], schedule_json: Optional[str] = None) -> Batch:
    lib = load()
    arr = (C.c_void_p * len(works))(*[w.handle for w in works])
    h = C.c_void_p()
    js = schedule_json.encode() if schedule_json else None
    _check(lib.sos_batch_setup(len(works), arr, js, C.byref(h)), None)
    return Batch(h, list(works))


def sos_batch_solve(batch: Batch) -> List[dict]:
    infos = (sos_info * len(batch.works))()
    _check(load().sos_batch_solve(batch.handle, infos), batch=batch.handle)
    return [i.as_dict() for i in infos]


def sos_batch_reset(batch: Batch) -> None:
    _check(load().sos_batch_reset(batch.handle), batch=batch.handle)


def sos_batch_last_ms(batch: Batch) -> float:
    return float(load().sos_batch_last_ms(batch.handle))


def sos_batch_phase_ms(batch: Batch, phase: int) -> float:
    return float(load().sos_batch_phase_ms(batch.handle, int(phase)))


def sos_batch_free(batch: Batch) -> None:
    batch.free()


# ---------------------------------------------------------------- learned warm start
def _dev(t):
    """Device pointer of a contiguous float32 cuda tensor."""
    import torch
    assert t.is_cuda and t.dtype == torch.float32 and t.is_contiguous()
    return C.c_void_p(t.data_ptr())


def sos_layout_size(w: Work) -> int:
    return int(load().sos_layout_size(w.handle))


def _check_rows(t, count: int, ld: int):
    if t.dim() != 2 or t.shape[0] < count or t.shape[1] != ld or t.stride(0) != ld:
        raise ValueError(f"expected a contiguous ({count}, {ld}) float32 cuda tensor, got {tuple(t.shape)}")


def sos_batch_warm_start(batch: Batch, pred, ld: int) -> None:
    """pred: cuda float32 tensor with one row of ld >= nx + m values per problem."""
    _check_rows(pred, len(batch.works), ld)
    _check(load().sos_batch_warm_start(batch.handle, _dev(pred), int(ld)), batch=batch.handle)


def sos_batch_export_solutions(batch: Batch, out, ld: int) -> None:
    _check_rows(out, len(batch.works), ld)
    _check(load().sos_batch_export_solutions(batch.handle, _dev(out), int(ld)), batch=batch.handle)


class MLP:
    """Handle of the device MLP (all compute in the library's kernels)."""

    def __init__(self, n_in: int, n_hidden: int, n_out: int, max_batch: int, stream=None):
        self.n_in, self.n_hidden, self.n_out, self.max_batch = n_in, n_hidden, n_out, max_batch
        h = C.c_void_p()
        st = stream if stream is not None else current_stream()
        _check(load().sos_mlp_create(n_in, n_hidden, n_out, max_batch, st, C.byref(h)), None)
        self.handle = h
        self.num_params = int(load().sos_mlp_num_params(h))

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass

    def free(self):
        if getattr(self, "handle", None):
            load().sos_mlp_free(self.handle)
            self.handle = None

    def set_params(self, params: np.ndarray) -> None:
        p = np.ascontiguousarray(params, dtype=np.float32)
        assert p.shape == (self.num_params,)
        _check(load().sos_mlp_set_params(self.handle, p.ctypes.data_as(C.POINTER(C.c_float))), None)

    def get_params(self) -> np.ndarray:
        p = np.empty(self.num_params, dtype=np.float32)
        _check(load().sos_mlp_get_params(self.handle, p.ctypes.data_as(C.POINTER(C.c_float))), None)
        return p

    def set_output_affine(self, scale: np.ndarray, shift: np.ndarray) -> None:
        s = np.ascontiguousarray(scale, dtype=np.float32)
        t = np.ascontiguousarray(shift, dtype=np.float32)
        _check(load().sos_mlp_set_output_affine(self.handle, s.ctypes.data_as(C.POINTER(C.c_float)),
                                                t.ctypes.data_as(C.POINTER(C.c_float))), None)

    def forward(self, X, Y, apply_output_affine: bool = False) -> None:
        _check(load().sos_mlp_forward(self.handle, _dev(X), X.shape[0], _dev(Y), int(apply_output_affine)), None)

    def gradient(self, X, T):
        g = np.empty(self.num_params, dtype=np.float32)
        loss = C.c_double()
        _check(load().sos_mlp_gradient(self.handle, _dev(X), _dev(T), X.shape[0],
                                       g.ctypes.data_as(C.POINTER(C.c_float)), C.byref(loss)), None)
        return g, loss.value

    def train_step_rows(self, X, T, rows, lr: float, want_loss: bool = False):
        """One Adam step on rows `rows` (a contiguous int32 cuda tensor) of X and T, gathered by the
        library."""
        import torch
        assert rows.is_cuda and rows.dtype == torch.int32 and rows.is_contiguous()
        assert X.shape[1] == self.n_in and T.shape[1] == self.n_out
        loss = C.c_double()
        _check(load().sos_mlp_train_step_rows(self.handle, _dev(X), _dev(T), C.c_void_p(rows.data_ptr()),
                                              int(rows.shape[0]), float(lr), C.byref(loss) if want_loss else None),
               None)
        return loss.value if want_loss else None

    def train_step(self, X, T, lr: float, want_loss: bool = False):
        loss = C.c_double()
        _check(load().sos_mlp_train_step(self.handle, _dev(X), _dev(T), X.shape[0], float(lr),
                                         C.byref(loss) if want_loss else None), None)
        return loss.value if want_loss else None
