"""Thin ctypes binding of ``liblor.so`` (the C ABI in include/lor.h).

Argument marshalling only: every step of the solver runs in the library's HIP
kernels.  Device vectors are torch tensors (float64, on the current device);
their ``data_ptr()`` and torch's current HIP stream are handed to the library.
Importing this module loads the library and raises if it is not built -- there
is no fallback.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liblor.so")

LOR_OK, LOR_EINVAL, LOR_EJACOBIAN, LOR_EPIVOT = 0, -1, -2, -3
LOR_EBREAKDOWN, LOR_ENOCONV, LOR_EHIP, LOR_ENOMEM, LOR_ESTATE = -4, -5, -6, -7, -8
LOR_EACCURACY = -9
LOR_CG, LOR_IP, LOR_BR2 = 0, 1, 2
LOR_BC_DIRICHLET, LOR_BC_NEUMANN = 0, 1
LOR_PREC_FP64, LOR_PREC_MIXED = 0, 1
LOR_ORD_MDF, LOR_ORD_NATURAL, LOR_ORD_RCM = 0, 1, 2
LOR_PROLONG_SUM, LOR_PROLONG_POU = 0, 1
LOR_PATCH_VERTEX, LOR_PATCH_SINGLE, LOR_PATCH_SLABS, LOR_PATCH_VERTEX_ISO = 0, 1, 2, 3
LOR_LAUNCH_AUTO, LOR_LAUNCH_VERTEX, LOR_LAUNCH_BUCKETS = 0, 1, 2
LOR_GEOM_STORED, LOR_GEOM_ONFLY = 0, 1
LOR_MAP_LDOF, LOR_MAP_ORDER, LOR_MAP_ORDER_OFFSET = 0, 1, 2
LOR_MAP_SCHEDULE, LOR_MAP_SCHEDULE_OFFSET, LOR_MAP_E2L = 3, 4, 5

EXPORTED = [
    "lor_default_options", "lor_error_string", "lor_setup", "lor_ndofs", "lor_device_bytes",
    "lor_dof_coords", "lor_assemble_rhs", "lor_apply_A", "lor_apply_P", "lor_pcg_solve",
    "lor_export_maps", "lor_export_stencils", "lor_gll", "lor_mdf_order", "lor_free",
    "lor_last_error_detail", "lor_timing", "lor_timing_read", "lor_pcg_solve_batch",
    "lor_nn_param_count", "lor_nn_create", "lor_nn_get_params", "lor_nn_shape", "lor_nn_patch_data",
    "lor_nn_forward", "lor_nn_gradients", "lor_nn_train_step", "lor_nn_attach", "lor_nn_free",
    "lor_bf16_gemm", "lor_apply_P_noalloc", "lor_noalloc_scratch_bytes", "lor_workspace_bytes",
    "lor_bind_workspace", "lor_element_coords", "lor_launch_order", "lor_f64_gemm", "lor_apply_P_batch",
]
LOR_NN_OFF, LOR_NN_REPLACE, LOR_NN_WARMSTART = 0, 1, 2
LOR_T_APPLY_A, LOR_T_PATCH, LOR_T_COARSE = 0, 1, 2


class LorError(RuntimeError):
    def __init__(self, code: int, where: str):
        self.code = code
        detail = (_lib.lor_last_error_detail().decode() if code in (LOR_EHIP, LOR_EINVAL, LOR_ENOMEM)
                  else "")
        super().__init__(f"{where}: {error_string(code)} ({code}) {detail}")


class lor_mesh_t(C.Structure):
    _fields_ = [("dim", C.c_int), ("n", C.c_int * 3), ("vertex_xyz", C.POINTER(C.c_double)),
                ("bc", C.c_int), ("coef", C.POINTER(C.c_double)), ("node_xyz", C.POINTER(C.c_double))]


class lor_options_t(C.Structure):
    _fields_ = [("precision", C.c_int), ("ordering", C.c_int), ("flexible", C.c_int),
                ("nthreads", C.c_int), ("prolong_weights", C.c_int), ("patch_mode", C.c_int),
                ("sweep_grid_rows", C.c_int), ("nslabs", C.c_int),
                ("deterministic", C.c_int), ("launch_order", C.c_int), ("operator_geometry", C.c_int),
                ("nn_fallback", C.c_int)]


class lor_solve_info_t(C.Structure):
    _fields_ = [("iters", C.c_int), ("status", C.c_int), ("rel_res", C.c_double),
                ("rel_res_true", C.c_double), ("t_solve", C.c_double), ("t_setup", C.c_double),
                ("replacements", C.c_int), ("fallback_iter", C.c_int)]


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is not built; run python -m paper_1908_07071_amd.build")
    # Load torch's HIP runtime first: the library's libamdhip64.so.7 dependency
    # then resolves to that already-loaded runtime, so device memory and streams
    # created by torch are valid in the library (one runtime per process).
    import torch  # noqa: F401
    lib = C.CDLL(LIB_PATH)
    vp, dp, i32p, i64p = C.c_void_p, C.POINTER(C.c_double), C.POINTER(C.c_int32), C.POINTER(C.c_int64)
    sig = {
        "lor_default_options": (C.c_int, [C.POINTER(lor_options_t)]),
        "lor_error_string": (C.c_char_p, [C.c_int]),
        "lor_setup": (C.c_int, [C.POINTER(lor_mesh_t), C.c_int, C.c_int, C.c_double,
                                C.POINTER(lor_options_t), vp, C.POINTER(vp)]),
        "lor_ndofs": (C.c_int, [vp, i64p]),
        "lor_device_bytes": (C.c_int, [vp, C.POINTER(C.c_size_t)]),
        "lor_workspace_bytes": (C.c_int, [vp, C.POINTER(C.c_size_t)]),
        "lor_element_coords": (C.c_int, [vp, dp]),
        "lor_launch_order": (C.c_int, [vp, C.POINTER(C.c_int), C.POINTER(C.c_double), C.POINTER(C.c_double)]),
        "lor_bind_workspace": (C.c_int, [vp, vp, C.c_size_t, vp]),
        "lor_dof_coords": (C.c_int, [vp, dp]),
        "lor_assemble_rhs": (C.c_int, [vp, vp, vp, vp]),
        "lor_apply_A": (C.c_int, [vp, vp, vp, vp]),
        "lor_apply_P": (C.c_int, [vp, vp, vp, vp]),
        "lor_apply_P_noalloc": (C.c_int, [vp, vp, vp, vp]),
        "lor_apply_P_batch": (C.c_int, [C.POINTER(vp), C.c_int, C.POINTER(vp), C.POINTER(vp), vp]),
        "lor_noalloc_scratch_bytes": (C.c_int, [vp, C.POINTER(C.c_size_t), C.POINTER(C.c_size_t)]),
        "lor_pcg_solve": (C.c_int, [vp, vp, vp, C.c_double, C.c_int, C.POINTER(lor_solve_info_t), vp]),
        "lor_export_maps": (C.c_int, [vp, C.c_int, i32p, i64p]),
        "lor_export_stencils": (C.c_int, [vp, C.c_int, dp, i64p]),
        "lor_gll": (C.c_int, [C.c_int, dp, dp]),
        "lor_mdf_order": (C.c_int, [C.c_int, i32p, dp, C.c_int, i32p, i32p, i32p, dp, dp]),
        "lor_free": (C.c_int, [vp]),
        "lor_last_error_detail": (C.c_char_p, []),
        "lor_timing": (C.c_int, [vp, C.c_int]),
        "lor_timing_read": (C.c_int, [vp, C.c_int, dp, i64p]),
        "lor_pcg_solve_batch": (C.c_int, [C.POINTER(vp), C.c_int, C.c_int, C.POINTER(vp), C.POINTER(vp),
                                          C.c_double, C.c_int, C.POINTER(lor_solve_info_t), vp]),
        "lor_nn_param_count": (C.c_int, [C.c_int, i64p]),
        "lor_nn_create": (C.c_int, [vp, C.c_int, dp, C.c_int, vp, C.POINTER(vp)]),
        "lor_nn_get_params": (C.c_int, [vp, dp]),
        "lor_nn_shape": (C.c_int, [vp, C.POINTER(C.c_int), C.POINTER(C.c_int)]),
        "lor_nn_patch_data": (C.c_int, [vp, vp, vp, vp, vp, vp]),
        "lor_nn_forward": (C.c_int, [vp, vp, C.c_int, vp, vp]),
        "lor_nn_gradients": (C.c_int, [vp, vp, vp, C.c_int, dp, dp, vp]),
        "lor_nn_train_step": (C.c_int, [vp, vp, vp, C.c_int, C.c_double, dp, vp]),
        "lor_nn_attach": (C.c_int, [vp, vp, C.c_int]),
        "lor_nn_free": (C.c_int, [vp]),
        "lor_bf16_gemm": (C.c_int, [C.c_int, C.c_int, C.c_int, vp, C.c_int64, C.c_int64, vp, C.c_int64,
                                    C.c_int64, vp, C.c_int64, vp]),
        "lor_f64_gemm": (C.c_int, [C.c_int, C.c_int, C.c_int, C.c_double, vp, C.c_int64, vp, C.c_int64,
                                   C.c_double, vp, C.c_int64, vp]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    return lib


_lib = _load()


def error_string(code: int) -> str:
    return _lib.lor_error_string(int(code)).decode()


def _check(rc: int, where: str):
    if rc != LOR_OK:
        raise LorError(rc, where)


def _dptr(a: np.ndarray):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _iptr(a: np.ndarray):
    return a.ctypes.data_as(C.POINTER(C.c_int32))


def _stream(stream):
    if stream is not None:
        return C.c_void_p(int(stream))
    import torch
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def _devt(t, dtype_name, name):
    import torch
    dt = getattr(torch, dtype_name)
    if not (isinstance(t, torch.Tensor) and t.is_cuda and t.dtype == dt and t.is_contiguous()):
        raise TypeError(f"{name} must be a contiguous {dtype_name} device tensor")
    return C.c_void_p(t.data_ptr())


def _dev(t, name):
    import torch
    if not (isinstance(t, torch.Tensor) and t.is_cuda and t.dtype == torch.float64 and t.is_contiguous()):
        raise TypeError(f"{name} must be a contiguous float64 device tensor")
    return C.c_void_p(t.data_ptr())


# ---------------------------------------------------------------- host-only

def lor_gll(p: int):
    x = np.zeros(p + 1)
    w = np.zeros(p + 1)
    _check(_lib.lor_gll(int(p), _dptr(x), _dptr(w)), "lor_gll")
    return x, w


def lor_mdf_order(dim: int, shape, rows: np.ndarray, natural: bool = False, ordering=None):
    """(order, level_ptr, L, D) of one patch matrix given as (n, 3^dim) stencil rows;
    ordering: LOR_ORD_* (default MDF, or natural order when natural is set)."""
    if ordering is None:
        ordering = LOR_ORD_NATURAL if natural else LOR_ORD_MDF
    m = np.ascontiguousarray(shape, dtype=np.int32)
    n = int(np.prod(m))
    ns = 3 ** dim
    rows = np.ascontiguousarray(rows, dtype=np.float64).reshape(n, ns)
    order = np.zeros(n, np.int32)
    lvl = np.zeros(n + 1, np.int32)
    depth = np.zeros(1, np.int32)
    L = np.zeros((n, ns))
    D = np.zeros(n)
    rc = _lib.lor_mdf_order(int(dim), _iptr(m), _dptr(rows), int(ordering), _iptr(order),
                            _iptr(lvl), _iptr(depth), _dptr(L), _dptr(D))
    _check(rc, "lor_mdf_order")
    return order, lvl[:int(depth[0]) + 1].copy(), L, D


# ---------------------------------------------------------------- handles

def lor_default_options():
    o = lor_options_t()
    _check(_lib.lor_default_options(C.byref(o)), "lor_default_options")
    return o


def lor_setup(dim: int, n, vertices: np.ndarray, p: int, method: int = LOR_CG, penalty: float = 0.0,
              options: lor_options_t | None = None, bc: int = LOR_BC_DIRICHLET, stream=None, coef=None,
              nodes=None):
    """Returns an opaque handle (ctypes void pointer).  coef: None or b at the
    elements' GLL nodes, n_el x (p+1)^dim values (E-vector layout).  nodes:
    None or the GLL-grid node coordinates of a curved mesh, ((n_i p + 1)...)
    x dim."""
    n = [int(n)] * dim if np.isscalar(n) else [int(v) for v in n]
    verts = np.ascontiguousarray(vertices, dtype=np.float64)
    mesh = lor_mesh_t()
    mesh.dim = dim
    for i in range(3):
        mesh.n[i] = n[i] if i < dim else 1
    mesh.vertex_xyz = _dptr(verts)
    mesh.bc = bc
    if coef is not None:
        cf = np.ascontiguousarray(coef, dtype=np.float64).ravel()
        if cf.size != int(np.prod(n)) * (p + 1) ** dim:
            raise ValueError("coef needs n_el * (p+1)^dim values")
        mesh.coef = _dptr(cf)
    if nodes is not None:
        nd = np.ascontiguousarray(nodes, dtype=np.float64)
        if nd.shape != (int(np.prod([v * p + 1 for v in n])), dim):
            raise ValueError("nodes needs (prod(n_i p + 1), dim) values")
        mesh.node_xyz = _dptr(nd)
    h = C.c_void_p()
    opt = C.byref(options) if options is not None else None
    rc = _lib.lor_setup(C.byref(mesh), int(p), int(method), float(penalty), opt, _stream(stream), C.byref(h))
    _check(rc, "lor_setup")
    return h


def lor_launch_order(h):
    """(order used, ms per patch launch in vertex order, in buckets)."""
    o, a, b = C.c_int(), C.c_double(), C.c_double()
    _check(_lib.lor_launch_order(h, C.byref(o), C.byref(a), C.byref(b)), "lor_launch_order")
    return o.value, a.value, b.value


def lor_ndofs(h) -> int:
    n = C.c_int64()
    _check(_lib.lor_ndofs(h, C.byref(n)), "lor_ndofs")
    return n.value


def lor_device_bytes(h) -> int:
    n = C.c_size_t()
    _check(_lib.lor_device_bytes(h, C.byref(n)), "lor_device_bytes")
    return n.value


def lor_workspace_bytes(h) -> int:
    n = C.c_size_t()
    _check(_lib.lor_workspace_bytes(h, C.byref(n)), "lor_workspace_bytes")
    return n.value


def lor_bind_workspace(h, ws, stream=None):
    """Moves the handle's device data into ``ws``, a contiguous device tensor
    (any dtype) of at least lor_workspace_bytes(h) bytes, 256-byte aligned,
    which must then outlive the handle and not be written by the caller."""
    import torch
    if not (isinstance(ws, torch.Tensor) and ws.is_cuda and ws.is_contiguous()):
        raise TypeError("ws must be a contiguous device tensor")
    nbytes = ws.numel() * ws.element_size()
    _check(_lib.lor_bind_workspace(h, C.c_void_p(ws.data_ptr()), C.c_size_t(nbytes), _stream(stream)),
           "lor_bind_workspace")


def lor_element_coords(h, dim: int, nel: int, p: int) -> np.ndarray:
    out = np.zeros((nel * (p + 1) ** dim, dim))
    _check(_lib.lor_element_coords(h, _dptr(out)), "lor_element_coords")
    return out


def lor_dof_coords(h, dim: int) -> np.ndarray:
    out = np.zeros((lor_ndofs(h), dim))
    _check(_lib.lor_dof_coords(h, _dptr(out)), "lor_dof_coords")
    return out


def lor_assemble_rhs(h, f, b, stream=None):
    _check(_lib.lor_assemble_rhs(h, _dev(f, "f"), _dev(b, "b"), _stream(stream)), "lor_assemble_rhs")


def lor_apply_A(h, x, y, stream=None):
    _check(_lib.lor_apply_A(h, _dev(x, "x"), _dev(y, "y"), _stream(stream)), "lor_apply_A")


def lor_apply_P(h, r, z, stream=None):
    _check(_lib.lor_apply_P(h, _dev(r, "r"), _dev(z, "z"), _stream(stream)), "lor_apply_P")


def lor_apply_P_noalloc(h, r, z, stream=None):
    _check(_lib.lor_apply_P_noalloc(h, _dev(r, "r"), _dev(z, "z"), _stream(stream)),
           "lor_apply_P_noalloc")


def lor_noalloc_scratch_bytes(h):
    need, cap = C.c_size_t(), C.c_size_t()
    _check(_lib.lor_noalloc_scratch_bytes(h, C.byref(need), C.byref(cap)), "lor_noalloc_scratch_bytes")
    return need.value, cap.value


def lor_pcg_solve(h, b, x, rtol: float = 1e-8, maxit: int = 1000, stream=None, check: bool = True):
    info = lor_solve_info_t()
    rc = _lib.lor_pcg_solve(h, _dev(b, "b"), _dev(x, "x"), float(rtol), int(maxit), C.byref(info),
                            _stream(stream))
    if check and rc not in (LOR_OK,):
        raise LorError(rc, "lor_pcg_solve")
    return info


def lor_apply_P_batch(handles, r, z, stream=None):
    """z[i] = B_i r[i] for every handle, patch corrections of like handles in
    one launch."""
    n = len(handles)
    if n == 0 or len(r) != n or len(z) != n:
        raise ValueError("one r and one z per handle")
    for i in range(n):
        m = lor_ndofs(handles[i])
        if r[i].numel() != m or z[i].numel() != m:
            raise ValueError(f"problem {i}: vectors must have {m} entries")
    hs = (C.c_void_p * n)(*[h.value for h in handles])
    rp = (C.c_void_p * n)(*[_dev(t, "r").value for t in r])
    zp = (C.c_void_p * n)(*[_dev(t, "z").value for t in z])
    _check(_lib.lor_apply_P_batch(hs, n, rp, zp, _stream(stream)), "lor_apply_P_batch")


def lor_pcg_solve_batch(handles, b, x, rtol: float = 1e-8, maxit: int = 1000, stream=None,
                        check: bool = True):
    """Batched solve: ``handles`` has one entry per problem; ``b`` and ``x`` are
    lists of nprob * nrhs device tensors, pair k = i * nrhs + j using
    handles[i].  Returns the list of per-pair solve infos."""
    nprob = len(handles)
    if nprob == 0 or len(b) != len(x) or len(b) % nprob:
        raise ValueError("b and x need nprob * nrhs tensors")
    nrhs = len(b) // nprob
    for k in range(len(b)):
        n = lor_ndofs(handles[k // nrhs])
        if b[k].numel() != n or x[k].numel() != n:
            raise ValueError(f"pair {k}: vectors must have {n} entries")
    hs = (C.c_void_p * nprob)(*[h.value for h in handles])
    bp = (C.c_void_p * len(b))(*[_dev(t, "b").value for t in b])
    xp = (C.c_void_p * len(x))(*[_dev(t, "x").value for t in x])
    infos = (lor_solve_info_t * len(b))()
    rc = _lib.lor_pcg_solve_batch(hs, nprob, nrhs, bp, xp, float(rtol), int(maxit), infos,
                                  _stream(stream))
    if check and rc != LOR_OK:
        raise LorError(rc, "lor_pcg_solve_batch")
    return list(infos)


def lor_export_maps(h, which: int) -> np.ndarray:
    n = C.c_int64()
    _check(_lib.lor_export_maps(h, int(which), None, C.byref(n)), "lor_export_maps")
    out = np.zeros(n.value, np.int32)
    _check(_lib.lor_export_maps(h, int(which), _iptr(out), C.byref(n)), "lor_export_maps")
    return out


def lor_export_stencils(h, level: int) -> np.ndarray:
    n = C.c_int64()
    _check(_lib.lor_export_stencils(h, int(level), None, C.byref(n)), "lor_export_stencils")
    out = np.zeros(n.value)
    _check(_lib.lor_export_stencils(h, int(level), _dptr(out), C.byref(n)), "lor_export_stencils")
    return out


def lor_free(h):
    if h is not None and h.value:
        _check(_lib.lor_free(h), "lor_free")
        h.value = None


def lor_timing(h, enable: bool):
    _check(_lib.lor_timing(h, int(bool(enable))), "lor_timing")


def lor_timing_read(h, which: int):
    """(total milliseconds, launches) of one kernel class since the last reset."""
    t = C.c_double()
    n = C.c_int64()
    _check(_lib.lor_timing_read(h, int(which), C.byref(t), C.byref(n)), "lor_timing_read")
    return t.value, n.value


# ---------------------------------------------------------------- learned patch correction

def lor_nn_param_count(channels: int) -> int:
    n = C.c_int64()
    _check(_lib.lor_nn_param_count(int(channels), C.byref(n)), "lor_nn_param_count")
    return n.value


def lor_nn_create(h, channels: int, params: np.ndarray, max_batch: int, stream=None):
    p = np.ascontiguousarray(params, dtype=np.float64)
    if p.size != lor_nn_param_count(channels):
        raise ValueError("parameter vector has the wrong length")
    nn = C.c_void_p()
    _check(_lib.lor_nn_create(h, int(channels), _dptr(p), int(max_batch), _stream(stream), C.byref(nn)),
           "lor_nn_create")
    nn._keep = p
    return nn


def lor_nn_get_params(nn, channels: int) -> np.ndarray:
    out = np.zeros(lor_nn_param_count(channels))
    _check(_lib.lor_nn_get_params(nn, _dptr(out)), "lor_nn_get_params")
    return out


def lor_nn_shape(nn):
    j, g = C.c_int(), C.c_int()
    _check(_lib.lor_nn_shape(nn, C.byref(j), C.byref(g)), "lor_nn_shape")
    return j.value, g.value


def lor_nn_patch_data(nn, r, X, T, scale, stream=None):
    _check(_lib.lor_nn_patch_data(nn, _dev(r, "r"), _devt(X, "float32", "X"), _devt(T, "float32", "T"),
                                  _dev(scale, "scale"), _stream(stream)), "lor_nn_patch_data")


def lor_nn_forward(nn, X, nb: int, Y, stream=None):
    _check(_lib.lor_nn_forward(nn, _devt(X, "float32", "X"), int(nb), _devt(Y, "float32", "Y"),
                               _stream(stream)), "lor_nn_forward")


def lor_nn_gradients(nn, X, T, nb: int, nparam: int, stream=None):
    loss = C.c_double()
    g = np.zeros(nparam)
    _check(_lib.lor_nn_gradients(nn, _devt(X, "float32", "X"), _devt(T, "float32", "T"), int(nb),
                                 C.byref(loss), _dptr(g), _stream(stream)), "lor_nn_gradients")
    return loss.value, g


def lor_nn_train_step(nn, X, T, nb: int, lr: float, stream=None) -> float:
    loss = C.c_double()
    _check(_lib.lor_nn_train_step(nn, _devt(X, "float32", "X"), _devt(T, "float32", "T"), int(nb),
                                  float(lr), C.byref(loss), _stream(stream)), "lor_nn_train_step")
    return loss.value


def lor_nn_attach(h, nn, mode: int):
    _check(_lib.lor_nn_attach(h, nn, int(mode)), "lor_nn_attach")


def lor_nn_free(nn):
    _check(_lib.lor_nn_free(nn), "lor_nn_free")


def lor_f64_gemm(m, n, k, alpha, A, lda, B, ldb, beta, Cmat, ldc, stream=None):
    """C = alpha A B + beta C on the device (row major, float64 tensors)."""
    _check(_lib.lor_f64_gemm(int(m), int(n), int(k), float(alpha), _dev(A, "A"), int(lda), _dev(B, "B"),
                             int(ldb), float(beta), _dev(Cmat, "C"), int(ldc), _stream(stream)),
           "lor_f64_gemm")


def lor_bf16_gemm(M, N, K, A, ai, ak, B, bk, bj, Cmat, ldc, stream=None):
    _check(_lib.lor_bf16_gemm(int(M), int(N), int(K), _devt(A, "int16", "A"), int(ai), int(ak),
                              _devt(B, "int16", "B"), int(bk), int(bj), _devt(Cmat, "float32", "C"),
                              int(ldc), _stream(stream)), "lor_bf16_gemm")
