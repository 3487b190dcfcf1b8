"""ctypes binding of libimrt (the C ABI declared in include/imrt.h).

Argument marshalling only: every function below calls the C entry point of
the same name.  Device buffers are passed as raw pointers (``Tensor.data_ptr()``
of CUDA/HIP tensors); the helper classes at the end manage handle lifetimes
and take PyTorch tensors.  Loading fails loudly when the HIP library has not
been built.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Optional

_HERE = os.path.dirname(os.path.abspath(__file__))
# IMRT_LIBRARY names another build of the same library (e.g. one compiled with
# different constants); by default the in-tree build is loaded.
LIB_PATH = os.environ.get("IMRT_LIBRARY") or os.path.join(_HERE, "libimrt.so")

# ---- error / status codes (imrt.h) ------------------------------------------
IMRT_OK, IMRT_EINVAL, IMRT_ENOMEM, IMRT_EHIP, IMRT_ENOTREADY, IMRT_EUNSUPPORTED, IMRT_ETIMEDOUT = (
    0, -1, -2, -3, -4, -5, -6)
IMRT_CONVERGED, IMRT_MAX_ITER, IMRT_STALLED, IMRT_LS_FAIL, IMRT_NUMERIC = 0, 1, 2, 3, 4
IMRT_F32, IMRT_BF16, IMRT_F16 = 0, 1, 2
STORAGE = {"f32": IMRT_F32, "bf16": IMRT_BF16, "f16": IMRT_F16}
STATUS_NAMES = {IMRT_CONVERGED: "converged", IMRT_MAX_ITER: "max_iter", IMRT_STALLED: "stalled",
                IMRT_LS_FAIL: "line_search_failed", IMRT_NUMERIC: "non_finite"}


class imrt_penalty(C.Structure):
    _fields_ = [("T_under", C.c_double), ("T_over", C.c_double),
                ("w_under", C.c_double), ("w_over", C.c_double)]


class imrt_geometry(C.Structure):
    _fields_ = [("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32), ("h", C.c_double),
                ("r_ptv", C.c_double), ("r_rectum", C.c_double), ("r_bladder", C.c_double),
                ("n_beams", C.c_int32), ("beamlet", C.c_double), ("sigma", C.c_double),
                ("tau", C.c_double), ("mu", C.c_double), ("margin", C.c_double),
                ("coarse_normal", C.c_int32)]


class imrt_solve_params(C.Structure):
    _fields_ = [("eps", C.c_double), ("alpha", C.c_double), ("lambda0", C.c_double),
                ("delta", C.c_double), ("max_iter", C.c_int32), ("max_backtracks", C.c_int32),
                ("fixed_iters", C.c_int32), ("trials_per_pass", C.c_int32), ("profile", C.c_int32),
                ("warm_start", C.c_int32), ("trace", C.c_void_p), ("resume", C.c_int32), ("k0", C.c_int32),
                ("G_prev", C.c_double), ("lambda_prev", C.c_double)]


class imrt_trace_entry(C.Structure):
    _fields_ = [("k", C.c_int32), ("backtracks", C.c_int32), ("lambda_", C.c_double),
                ("step_sq", C.c_double), ("G", C.c_double)]


class imrt_solve_result(C.Structure):
    _fields_ = [("iterations", C.c_int32), ("forward_passes", C.c_int32),
                ("adjoint_passes", C.c_int32), ("status", C.c_int32), ("G_initial", C.c_double),
                ("G_final", C.c_double), ("device_ms", C.c_double), ("forward_kernel_ms", C.c_double),
                ("adjoint_kernel_ms", C.c_double)]


class imrt_request(C.Structure):
    _fields_ = [("patient", C.c_int64), ("geometry", C.POINTER(imrt_geometry)), ("storage", C.c_int),
                ("penalties", C.POINTER(imrt_penalty)), ("nstruct", C.c_int32), ("x0", C.c_double),
                ("params", imrt_solve_params)]


class imrt_serve_times(C.Structure):
    _fields_ = [("queue_ms", C.c_double), ("plan_ms", C.c_double), ("lambda0", C.c_double),
                ("nnz", C.c_int64), ("nv", C.c_int32), ("nb", C.c_int32)]


_vp = C.c_void_p
_i32p = C.POINTER(C.c_int32)
_f32p = C.POINTER(C.c_float)
_u8p = C.POINTER(C.c_uint8)
_dp = C.POINTER(C.c_double)
_u16p = C.POINTER(C.c_uint16)

# name -> (restype, argtypes); one entry per function of include/imrt.h
SIGNATURES = {
    "imrt_ctx_create": (C.c_int, [C.c_int, _vp, C.POINTER(_vp)]),
    "imrt_ctx_destroy": (C.c_int, [_vp]),
    "imrt_ctx_stream": (C.c_int, [_vp, C.POINTER(_vp)]),
    "imrt_ctx_set_option": (C.c_int, [_vp, C.c_char_p, C.c_int64]),
    "imrt_ctx_get_option": (C.c_int, [_vp, C.c_char_p, C.POINTER(C.c_int64)]),
    "imrt_build_dose_matrix": (C.c_int, [_vp, C.POINTER(imrt_geometry), C.c_int, C.POINTER(_vp), _u8p]),
    "imrt_dose_from_csr": (C.c_int, [_vp, C.c_int32, C.c_int32, C.c_int64, _i32p, _i32p, _f32p, C.c_int,
                                     C.POINTER(_vp)]),
    "imrt_dose_info": (C.c_int, [_vp, _i32p, _i32p, C.POINTER(C.c_int64)]),
    "imrt_read_probe": (C.c_int, [_vp, _vp, C.c_int64, C.c_int32, C.POINTER(C.c_double)]),
    "imrt_dose_export": (C.c_int, [_vp, _i32p, _i32p, _f32p, _i32p, _i32p, _f32p, _u8p]),
    "imrt_dose_export_codes": (C.c_int, [_vp, _u16p, _u16p, _f32p]),
    "imrt_dose_storage": (C.c_int, [_vp, _i32p]),
    "imrt_dose_apply": (C.c_int, [_vp, _vp, _vp]),
    "imrt_dose_apply_transpose": (C.c_int, [_vp, _vp, _vp]),
    "imrt_dose_destroy": (C.c_int, [_vp]),
    "imrt_plan_create": (C.c_int, [_vp, _vp, C.POINTER(_vp)]),
    "imrt_set_structures": (C.c_int, [_vp, _u8p, C.c_int32]),
    "imrt_set_penalties": (C.c_int, [_vp, C.POINTER(imrt_penalty)]),
    "imrt_set_voxel_targets": (C.c_int, [_vp, _f32p, _f32p]),
    "imrt_evaluate_objective": (C.c_int, [_vp, _vp, _dp, _vp]),
    "imrt_gradient": (C.c_int, [_vp, _vp, _vp, _dp]),
    "imrt_gradient_noalloc": (C.c_int, [_vp, _vp, _vp, _dp]),
    "imrt_project": (C.c_int, [_vp, _vp, _vp, C.c_double, _vp, _dp]),
    "imrt_estimate_lambda0": (C.c_int, [_vp, _vp, C.c_int32, _dp, _dp]),
    "imrt_solve": (C.c_int, [_vp, C.POINTER(imrt_solve_params), _vp, C.POINTER(imrt_solve_result)]),
    "imrt_solve_batch": (C.c_int, [C.c_int32, C.POINTER(_vp), C.POINTER(imrt_solve_params), C.POINTER(_vp),
                                   C.POINTER(imrt_solve_result)]),
    "imrt_dose_repartition": (C.c_int, [_vp, C.c_int32, C.c_int32]),
    "imrt_dose_partition": (C.c_int, [_vp, _i32p, _i32p]),
    "imrt_dose_repartition_targets": (C.c_int, [_vp, C.c_int32, C.c_int32]),
    "imrt_batch_autotune": (C.c_int, [C.c_int32, C.POINTER(_vp), C.POINTER(imrt_solve_params), C.POINTER(_vp),
                                      C.c_int32, _i32p, _i32p]),
    "imrt_plan_destroy": (C.c_int, [_vp]),
    "imrt_server_create": (C.c_int, [_vp, C.c_int64, C.c_int32, C.POINTER(_vp)]),
    "imrt_server_submit": (C.c_int, [_vp, C.POINTER(imrt_request), C.POINTER(C.c_int64)]),
    "imrt_server_wait": (C.c_int, [_vp, C.c_int64, _f32p, C.c_int32, C.POINTER(imrt_solve_result),
                                   C.POINTER(imrt_serve_times), C.c_int64]),
    "imrt_server_stats": (C.c_int, [_vp, C.POINTER(C.c_int64), C.POINTER(C.c_int64), C.POINTER(C.c_int64),
                                    C.POINTER(C.c_int64)]),
    "imrt_server_adjoint_groups": (C.c_int, [_vp, C.POINTER(C.c_int64), C.POINTER(C.c_int64)]),
    "imrt_server_destroy": (C.c_int, [_vp]),
    "imrt_last_error": (C.c_char_p, []),
}

_lib = None


def load(path: str = LIB_PATH) -> C.CDLL:
    """Load libimrt.so and bind every entry point (raises if it is not built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"{path} is missing: build it with `python -m paper_0908_4421_amd.build`")
    lib = C.CDLL(path)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


class ImrtError(RuntimeError):
    def __init__(self, code: int, func: str, msg: str):
        super().__init__(f"{func} failed ({code}): {msg}")
        self.code = code


def _check(code: int, func: str):
    if code != IMRT_OK:
        raise ImrtError(code, func, last_error())
    return code


def last_error() -> str:
    return load().imrt_last_error().decode(errors="replace")


def _ptr(t) -> Optional[int]:
    return None if t is None else t.data_ptr()


def _host(arr, ctype):
    return None if arr is None else arr.ctypes.data_as(C.POINTER(ctype))


# ---- raw entry points (same names as the C ABI) --------------------------------
def imrt_ctx_create(device: int, hip_stream: Optional[int]):
    out = _vp()
    _check(load().imrt_ctx_create(device, hip_stream, C.byref(out)), "imrt_ctx_create")
    return out


def imrt_ctx_destroy(ctx):
    return _check(load().imrt_ctx_destroy(ctx), "imrt_ctx_destroy")


def imrt_ctx_stream(ctx) -> int:
    out = _vp()
    _check(load().imrt_ctx_stream(ctx, C.byref(out)), "imrt_ctx_stream")
    return out.value or 0


def imrt_ctx_set_option(ctx, name: str, value: int):
    return _check(load().imrt_ctx_set_option(ctx, name.encode(), int(value)), "imrt_ctx_set_option")


def imrt_ctx_get_option(ctx, name: str) -> int:
    out = C.c_int64()
    _check(load().imrt_ctx_get_option(ctx, name.encode(), C.byref(out)), "imrt_ctx_get_option")
    return out.value


def imrt_build_dose_matrix(ctx, geom: imrt_geometry, storage: int = IMRT_F32, voxel_struct_out=None):
    out = _vp()
    _check(load().imrt_build_dose_matrix(ctx, C.byref(geom), storage, C.byref(out),
                                         _host(voxel_struct_out, C.c_uint8)), "imrt_build_dose_matrix")
    return out


def imrt_dose_from_csr(ctx, nv, nb, nnz, row_ptr, col_idx, val, storage: int = IMRT_F32):
    out = _vp()
    _check(load().imrt_dose_from_csr(ctx, nv, nb, nnz, _host(row_ptr, C.c_int32), _host(col_idx, C.c_int32),
                                     _host(val, C.c_float), storage, C.byref(out)), "imrt_dose_from_csr")
    return out


def imrt_read_probe(ctx, buf_ptr: int, nbytes: int, reps: int = 5) -> float:
    """GB/s of the best of `reps` streaming reads of a device buffer."""
    out = C.c_double()
    _check(load().imrt_read_probe(ctx, C.c_void_p(buf_ptr), nbytes, reps, C.byref(out)), "imrt_read_probe")
    return out.value


def imrt_dose_info(dose):
    nv, nb, nnz = C.c_int32(), C.c_int32(), C.c_int64()
    _check(load().imrt_dose_info(dose, C.byref(nv), C.byref(nb), C.byref(nnz)), "imrt_dose_info")
    return nv.value, nb.value, nnz.value


def imrt_dose_export(dose, row_ptr=None, col_idx=None, val=None, col_ptr=None, row_idx=None, cval=None,
                     voxel_struct=None):
    return _check(load().imrt_dose_export(dose, _host(row_ptr, C.c_int32), _host(col_idx, C.c_int32),
                                          _host(val, C.c_float), _host(col_ptr, C.c_int32),
                                          _host(row_idx, C.c_int32), _host(cval, C.c_float),
                                          _host(voxel_struct, C.c_uint8)), "imrt_dose_export")


def imrt_dose_export_codes(dose, val_code=None, cval_code=None, col_scale=None):
    return _check(load().imrt_dose_export_codes(dose, _host(val_code, C.c_uint16), _host(cval_code, C.c_uint16),
                                                _host(col_scale, C.c_float)), "imrt_dose_export_codes")


def imrt_dose_storage(dose) -> int:
    out = C.c_int32()
    _check(load().imrt_dose_storage(dose, C.byref(out)), "imrt_dose_storage")
    return out.value


def imrt_solve_batch(n: int, plans, params, x_devs, results):
    """plans: array of n plan handles; params: array of n imrt_solve_params;
    x_devs: array of n device pointers; results: array of n imrt_solve_result."""
    return _check(load().imrt_solve_batch(n, plans, params, x_devs, results), "imrt_solve_batch")


def imrt_dose_repartition(dose, adj_min_nnz: int, fwd_blocks_per_wave: int):
    return _check(load().imrt_dose_repartition(dose, int(adj_min_nnz), int(fwd_blocks_per_wave)),
                  "imrt_dose_repartition")


def imrt_dose_partition(dose):
    a, b = C.c_int32(), C.c_int32()
    _check(load().imrt_dose_partition(dose, C.byref(a), C.byref(b)), "imrt_dose_partition")
    return a.value, b.value


def imrt_dose_repartition_targets(dose, adj_workgroups: int, fwd_workgroups: int):
    return _check(load().imrt_dose_repartition_targets(dose, int(adj_workgroups), int(fwd_workgroups)),
                  "imrt_dose_repartition_targets")


def imrt_batch_autotune(n: int, plans, params, x_devs, tune_iters: int):
    a, b = C.c_int32(), C.c_int32()
    _check(load().imrt_batch_autotune(n, plans, params, x_devs, int(tune_iters), C.byref(a), C.byref(b)),
           "imrt_batch_autotune")
    return a.value, b.value


def imrt_server_create(ctx, budget_bytes: int, max_live: int):
    out = _vp()
    _check(load().imrt_server_create(ctx, int(budget_bytes), int(max_live), C.byref(out)), "imrt_server_create")
    return out


def imrt_server_submit(server, request: "imrt_request") -> int:
    t = C.c_int64()
    _check(load().imrt_server_submit(server, C.byref(request), C.byref(t)), "imrt_server_submit")
    return t.value


def imrt_server_wait(server, ticket: int, x_out=None, nb: int = 0, timeout_ms: int = 120000):
    res, times = imrt_solve_result(), imrt_serve_times()
    _check(load().imrt_server_wait(server, int(ticket), _host(x_out, C.c_float), int(nb), C.byref(res),
                                   C.byref(times), int(timeout_ms)), "imrt_server_wait")
    return res, times


def imrt_server_stats(server):
    v = [C.c_int64() for _ in range(4)]
    _check(load().imrt_server_stats(server, *[C.byref(x) for x in v]), "imrt_server_stats")
    return dict(zip(("used_bytes", "peak_bytes", "resident_matrices", "served"), (x.value for x in v)))


def imrt_server_adjoint_groups(server):
    shared, total = C.c_int64(), C.c_int64()
    _check(load().imrt_server_adjoint_groups(server, C.byref(shared), C.byref(total)), "imrt_server_adjoint_groups")
    return shared.value, total.value


def imrt_server_destroy(server):
    return _check(load().imrt_server_destroy(server), "imrt_server_destroy")


def imrt_dose_apply(dose, x_dev: int, d_dev: int):
    return _check(load().imrt_dose_apply(dose, x_dev, d_dev), "imrt_dose_apply")


def imrt_dose_apply_transpose(dose, r_dev: int, y_dev: int):
    return _check(load().imrt_dose_apply_transpose(dose, r_dev, y_dev), "imrt_dose_apply_transpose")


def imrt_dose_destroy(dose):
    return _check(load().imrt_dose_destroy(dose), "imrt_dose_destroy")


def imrt_plan_create(ctx, dose):
    out = _vp()
    _check(load().imrt_plan_create(ctx, dose, C.byref(out)), "imrt_plan_create")
    return out


def imrt_set_structures(plan, voxel_struct, nstruct: int):
    return _check(load().imrt_set_structures(plan, _host(voxel_struct, C.c_uint8), nstruct), "imrt_set_structures")


def imrt_set_penalties(plan, table):
    arr = (imrt_penalty * len(table))(*[imrt_penalty(*p) for p in table])
    return _check(load().imrt_set_penalties(plan, arr), "imrt_set_penalties")


def imrt_set_voxel_targets(plan, T_under, T_over):
    return _check(load().imrt_set_voxel_targets(plan, _host(T_under, C.c_float), _host(T_over, C.c_float)),
                  "imrt_set_voxel_targets")


def imrt_evaluate_objective(plan, x_dev: int, dose_dev: Optional[int] = None) -> float:
    G = C.c_double()
    _check(load().imrt_evaluate_objective(plan, x_dev, C.byref(G), dose_dev), "imrt_evaluate_objective")
    return G.value


def imrt_gradient(plan, x_dev: int, g_dev: int) -> float:
    G = C.c_double()
    _check(load().imrt_gradient(plan, x_dev, g_dev, C.byref(G)), "imrt_gradient")
    return G.value


def imrt_gradient_noalloc(plan, x_dev: int, g_dev: int, want_G: bool = True) -> Optional[float]:
    """imrt_gradient through the library's per-device static scratch (no
    device allocation); with want_G False nothing is copied back."""
    G = C.c_double()
    _check(load().imrt_gradient_noalloc(plan, x_dev, g_dev, C.byref(G) if want_G else None),
           "imrt_gradient_noalloc")
    return G.value if want_G else None


def imrt_project(plan, x_dev: int, g_dev: int, lam: float, x_out_dev: int) -> float:
    s = C.c_double()
    _check(load().imrt_project(plan, x_dev, g_dev, lam, x_out_dev, C.byref(s)), "imrt_project")
    return s.value


def imrt_estimate_lambda0(plan, v0_dev: int, iters: int):
    lam, sig = C.c_double(), C.c_double()
    _check(load().imrt_estimate_lambda0(plan, v0_dev, iters, C.byref(lam), C.byref(sig)), "imrt_estimate_lambda0")
    return lam.value, sig.value


def imrt_solve(plan, params: imrt_solve_params, x_dev: int) -> imrt_solve_result:
    res = imrt_solve_result()
    _check(load().imrt_solve(plan, C.byref(params), x_dev, C.byref(res)), "imrt_solve")
    return res


def imrt_plan_destroy(plan):
    return _check(load().imrt_plan_destroy(plan), "imrt_plan_destroy")


def imrt_last_error() -> str:
    return last_error()


# ---- helpers over the raw entry points ------------------------------------------
class Context:
    """A library context on ``device``, enqueuing on PyTorch's current stream."""

    def __init__(self, device: int = 0, stream: Optional[int] = None, **options):
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("libimrt needs a HIP GPU; none is visible")
        torch.cuda.set_device(device)
        if stream is None:
            stream = torch.cuda.current_stream(device).cuda_stream
        self.device = device
        self.handle = imrt_ctx_create(device, stream)
        for name, value in options.items():
            imrt_ctx_set_option(self.handle, name, value)

    def set_option(self, name: str, value: int):
        imrt_ctx_set_option(self.handle, name, value)

    def get_option(self, name: str) -> int:
        return imrt_ctx_get_option(self.handle, name)

    def close(self):
        if self.handle:
            imrt_ctx_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Dose:
    """A device-resident dose-deposition matrix (CSR + CSC)."""

    def __init__(self, ctx: Context, handle):
        self.ctx = ctx
        self.handle = handle
        self.nv, self.nb, self.nnz = imrt_dose_info(handle)
        self.storage = imrt_dose_storage(handle)

    @staticmethod
    def from_geometry(ctx: Context, spec, storage: str = "f32") -> "Dose":
        g = geometry_of(spec)
        return Dose(ctx, imrt_build_dose_matrix(ctx.handle, g, STORAGE[storage]))

    @staticmethod
    def from_csr(ctx: Context, nv, nb, row_ptr, col_idx, val, storage: str = "f32") -> "Dose":
        import numpy as np
        row_ptr = np.ascontiguousarray(row_ptr, dtype=np.int32)
        col_idx = np.ascontiguousarray(col_idx, dtype=np.int32)
        val = np.ascontiguousarray(val, dtype=np.float32)
        return Dose(ctx, imrt_dose_from_csr(ctx.handle, nv, nb, int(row_ptr[-1]), row_ptr, col_idx, val,
                                            STORAGE[storage]))

    def repartition(self, adj_min_nnz: int, fwd_blocks_per_wave: int):
        imrt_dose_repartition(self.handle, adj_min_nnz, fwd_blocks_per_wave)

    def partition(self):
        return imrt_dose_partition(self.handle)

    def repartition_targets(self, adj_workgroups: int, fwd_workgroups: int):
        """Per-plan partition targets (the batch search's and the server's rule)."""
        imrt_dose_repartition_targets(self.handle, adj_workgroups, fwd_workgroups)

    def export_codes(self):
        """16-bit storage: codes in CSR and CSC order and the beamlet scales."""
        import numpy as np
        q = np.empty(self.nnz, np.uint16)
        cq = np.empty(self.nnz, np.uint16)
        sc = np.empty(self.nb, np.float32)
        imrt_dose_export_codes(self.handle, q, cq, sc)
        return dict(val_code=q, cval_code=cq, col_scale=sc)

    def export(self, structures: bool = False):
        import numpy as np
        rp = np.empty(self.nv + 1, np.int32)
        ci = np.empty(self.nnz, np.int32)
        v = np.empty(self.nnz, np.float32)
        cp = np.empty(self.nb + 1, np.int32)
        ri = np.empty(self.nnz, np.int32)
        cv = np.empty(self.nnz, np.float32)
        sid = np.empty(self.nv, np.uint8) if structures else None
        imrt_dose_export(self.handle, rp, ci, v, cp, ri, cv, sid)
        return dict(row_ptr=rp, col_idx=ci, val=v, col_ptr=cp, row_idx=ri, cval=cv, struct_id=sid)

    def apply(self, x, out=None):
        import torch
        out = torch.empty(self.nv, dtype=torch.float32, device=x.device) if out is None else out
        imrt_dose_apply(self.handle, x.data_ptr(), out.data_ptr())
        return out

    def apply_transpose(self, r, out=None):
        import torch
        out = torch.empty(self.nb, dtype=torch.float32, device=r.device) if out is None else out
        imrt_dose_apply_transpose(self.handle, r.data_ptr(), out.data_ptr())
        return out

    def close(self):
        if self.handle:
            imrt_dose_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Plan:
    """Dose matrix + structures + penalties; objective, gradient, projection, solve."""

    def __init__(self, ctx: Context, dose: Dose):
        self.ctx = ctx
        self.dose = dose
        self.handle = imrt_plan_create(ctx.handle, dose.handle)

    def set_structures(self, voxel_struct, nstruct: int):
        import numpy as np
        arr = None if voxel_struct is None else np.ascontiguousarray(voxel_struct, dtype=np.uint8)
        imrt_set_structures(self.handle, arr, nstruct)

    def set_penalties(self, table):
        rows = [tuple(float(v) for v in row) for row in table]
        imrt_set_penalties(self.handle, rows)

    def set_voxel_targets(self, T_under, T_over):
        import numpy as np
        if T_under is None:
            imrt_set_voxel_targets(self.handle, None, None)
        else:
            imrt_set_voxel_targets(self.handle, np.ascontiguousarray(T_under, np.float32),
                                   np.ascontiguousarray(T_over, np.float32))

    def objective(self, x, dose_out=None) -> float:
        return imrt_evaluate_objective(self.handle, x.data_ptr(), _ptr(dose_out))

    def gradient(self, x, g=None):
        import torch
        g = torch.empty(self.dose.nb, dtype=torch.float32, device=x.device) if g is None else g
        G = imrt_gradient(self.handle, x.data_ptr(), g.data_ptr())
        return g, G

    def gradient_noalloc(self, x, g, want_G: bool = True):
        """Gradient into the caller's g through the allocation-free entry point."""
        return imrt_gradient_noalloc(self.handle, x.data_ptr(), g.data_ptr(), want_G)

    def project(self, x, g, lam: float, out=None):
        import torch
        out = torch.empty_like(x) if out is None else out
        s = imrt_project(self.handle, x.data_ptr(), g.data_ptr(), lam, out.data_ptr())
        return out, s

    def lambda0(self, v0, iters: int = 50):
        return imrt_estimate_lambda0(self.handle, v0.data_ptr(), iters)

    @staticmethod
    def solve_batch(plans, xs, *, eps, alpha, lambda0s, delta=1e-5, max_iter=20000, max_backtracks=60,
                    fixed_iters=False, trials_per_pass=1, trace=False, warm_start=False):
        """imrt_solve_batch over `plans` (list of Plan) from the device tensors
        `xs`; one lambda_0 per plan.  Returns [(result, trace or None)]."""
        n = len(plans)
        bufs = [(imrt_trace_entry * max(max_iter, 1))() if trace else None for _ in range(n)]
        params = (imrt_solve_params * n)(*[
            imrt_solve_params(eps, alpha, lam, delta, max_iter, max_backtracks, int(bool(fixed_iters)),
                              trials_per_pass, 0, int(bool(warm_start)), C.cast(b, C.c_void_p) if trace else None)
            for lam, b in zip(lambda0s, bufs)])
        handles = (_vp * n)(*[p.handle for p in plans])
        xptr = (_vp * n)(*[x.data_ptr() for x in xs])
        res = (imrt_solve_result * n)()
        imrt_solve_batch(n, handles, params, xptr, res)
        out = []
        for i in range(n):
            tr = None
            if trace:
                b = bufs[i]
                tr = [(b[j].k, b[j].backtracks, b[j].lambda_, b[j].step_sq, b[j].G)
                      for j in range(min(res[i].iterations, max_iter))]
            out.append((res[i], tr))
        return out

    @staticmethod
    def autotune_batch(plans, xs, *, eps, alpha, lambda0s, delta=1e-5, max_backtracks=60, trials_per_pass=1,
                       tune_iters=40, max_iter=20000):
        """imrt_batch_autotune: returns the per-plan targets (adjoint
        workgroups, forward workgroups) of the partition left applied.
        tune_iters > 0 times that many fixed iterations per candidate, 0 the
        whole batch solved to the stopping rule (max_iter cap)."""
        n = len(plans)
        it, fixed = (tune_iters, 1) if tune_iters > 0 else (max_iter, 0)
        params = (imrt_solve_params * n)(*[
            imrt_solve_params(eps, alpha, lam, delta, it, max_backtracks, fixed, trials_per_pass, 0, 0, None)
            for lam in lambda0s])
        handles = (_vp * n)(*[p.handle for p in plans])
        xptr = (_vp * n)(*[x.data_ptr() for x in xs])
        return imrt_batch_autotune(n, handles, params, xptr, tune_iters)

    def solve(self, x, *, eps, alpha, lambda0, delta=1e-5, max_iter=20000, max_backtracks=60,
              fixed_iters=False, trials_per_pass=1, trace=False, profile=0, warm_start=False, resume=None):
        """imrt_solve from the device tensor x (updated in place).  resume:
        None for a fresh start, else (k0, G_prev, lambda_prev) of the solve x
        comes from.  Returns (result, trace as (k, backtracks, lambda,
        step_sq, G) tuples or None)."""
        buf = (imrt_trace_entry * max(max_iter, 1))() if trace else None
        p = imrt_solve_params(eps, alpha, lambda0, delta, max_iter, max_backtracks, int(bool(fixed_iters)),
                              trials_per_pass, int(profile), int(bool(warm_start)),
                              C.cast(buf, C.c_void_p) if trace else None)
        if resume is not None:
            p.resume = 1
            p.k0, p.G_prev, p.lambda_prev = int(resume[0]), float(resume[1]), float(resume[2])
        res = imrt_solve(self.handle, p, x.data_ptr())
        tr = None
        if trace:
            tr = [(buf[i].k, buf[i].backtracks, buf[i].lambda_, buf[i].step_sq, buf[i].G)
                  for i in range(min(res.iterations, max_iter))]
        return res, tr

    def close(self):
        if self.handle:
            imrt_plan_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Server:
    """The re-plan server (imrt_server_*): submit requests from any thread,
    wait for their plans."""

    def __init__(self, ctx: "Context", budget_bytes: int, max_live: int = 64):
        self.ctx = ctx
        self.handle = imrt_server_create(ctx.handle, budget_bytes, max_live)
        self._traces = {}   # ticket -> trace buffer, kept alive until its wait

    def submit(self, patient: int, spec, table, *, storage="f32", x0=1.0, eps=1e-4, alpha=2.0, lambda0=0.0,
               delta=1e-5, max_iter=20000, max_backtracks=60, fixed_iters=False, trials_per_pass=1,
               warm_start=False, trace=False) -> int:
        """spec: a PhantomSpec building the patient's matrix when it is not
        resident (None to require a resident one); table: (nstruct, 4).
        trace: the plan's accepted iterations come back from wait()."""
        rows = [imrt_penalty(*[float(v) for v in row]) for row in table]
        pen = (imrt_penalty * len(rows))(*rows)
        geom = geometry_of(spec) if spec is not None else None
        buf = (imrt_trace_entry * max(max_iter, 1))() if trace else None
        req = imrt_request(int(patient), C.pointer(geom) if geom is not None else None, STORAGE[storage], pen,
                           len(rows), float(x0),
                           imrt_solve_params(eps, alpha, lambda0, delta, max_iter, max_backtracks,
                                             int(bool(fixed_iters)), trials_per_pass, 0, int(bool(warm_start)),
                                             C.cast(buf, C.c_void_p) if trace else None))
        ticket = imrt_server_submit(self.handle, req)
        if trace:
            self._traces[ticket] = (buf, max_iter)
        return ticket

    def trace_of(self, ticket: int, iterations: int):
        """The trace of a waited-on ticket submitted with trace=True, as
        (k, backtracks, lambda, step_sq, G) tuples."""
        buf, cap = self._traces.pop(ticket)
        return [(buf[i].k, buf[i].backtracks, buf[i].lambda_, buf[i].step_sq, buf[i].G)
                for i in range(min(iterations, cap))]

    def wait(self, ticket: int, nb: int = 0, timeout_s: float = 120.0):
        """(result, times, x as a numpy array or None when nb == 0).  Raises
        ImrtError with code IMRT_ETIMEDOUT when the plan is not ready within
        timeout_s seconds (the ticket stays pending)."""
        import numpy as np
        x = np.empty(nb, np.float32) if nb else None
        res, times = imrt_server_wait(self.handle, ticket, x, nb, max(1, int(timeout_s * 1e3)))
        return res, times, x

    def stats(self):
        st = imrt_server_stats(self.handle)
        st["adjoint_groups_shared"], st["adjoint_groups"] = imrt_server_adjoint_groups(self.handle)
        return st

    def close(self):
        if self.handle:
            imrt_server_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def geometry_of(spec) -> imrt_geometry:
    """imrt_geometry from a workload PhantomSpec (duck-typed)."""
    return imrt_geometry(spec.nx, spec.ny, spec.nz, spec.h, spec.r_ptv, spec.r_rectum, spec.r_bladder,
                         spec.n_beams, spec.beamlet, spec.sigma, spec.tau, spec.mu, spec.margin,
                         1 if getattr(spec, "coarse_normal", False) else 0)
