"""Thin Python binding of the C ABI in ``include/bte.h`` (ctypes).

Argument marshalling only: every step of the solver runs in the HIP library
``libbte.so``.  The library must have been built (``python -m
paper_1401_6047_amd.build``); importing this module without it raises.
PyTorch provides the device workspace and the stream.
"""
from __future__ import annotations

import ctypes
import os
import re
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libbte.so")
HEADER_PATH = os.path.join(os.path.dirname(_HERE), "include", "bte.h")

BTE_OK, BTE_EINVAL, BTE_ENOMEM, BTE_EDEVICE, BTE_EUNSTABLE, BTE_ESTATE = 0, -1, -2, -3, -4, -5
BTE_FP64, BTE_FP32_BULK = 0, 1
BTE_KERNEL_FUSED, BTE_KERNEL_TWO_PASS, BTE_KERNEL_FUSED2, BTE_KERNEL_FUSED3 = 0, 1, 2, 3
BTE_BATCH_PERSISTENT, BTE_BATCH_WIDE = 0, 1
STATUS_NAMES = {0: "BTE_OK", -1: "BTE_EINVAL", -2: "BTE_ENOMEM", -3: "BTE_EDEVICE",
                -4: "BTE_EUNSTABLE", -5: "BTE_ESTATE"}


class bte_grid(ctypes.Structure):
    _fields_ = [("n_x", ctypes.c_int32), ("n_y", ctypes.c_int32),
                ("phiy_min", ctypes.c_double), ("phiy_max", ctypes.c_double)]


class bte_params(ctypes.Structure):
    _fields_ = [("E_dc", ctypes.c_double), ("E_w", ctypes.c_double),
                ("omega", ctypes.c_double), ("B", ctypes.c_double),
                ("mu", ctypes.c_double), ("alpha", ctypes.c_double),
                ("tau", ctypes.c_double), ("dt", ctypes.c_double),
                ("precision", ctypes.c_int32), ("flags", ctypes.c_uint32)]


class bte_tuning(ctypes.Structure):
    _fields_ = [("kernel", ctypes.c_int32), ("rows_per_wave", ctypes.c_int32),
                ("waves_per_block", ctypes.c_int32), ("graph_steps", ctypes.c_int32)]


class bte_obs(ctypes.Structure):
    _fields_ = [("step", ctypes.c_int64), ("t", ctypes.c_double),
                ("v_dr", ctypes.c_double), ("norm", ctypes.c_double),
                ("n_avg", ctypes.c_int64), ("S_v", ctypes.c_double),
                ("S_vc", ctypes.c_double), ("v_avg", ctypes.c_double),
                ("absorption", ctypes.c_double), ("S_c", ctypes.c_double),
                ("absorption_cov", ctypes.c_double), ("edge_mass", ctypes.c_double),
                ("top_harm_mass", ctypes.c_double), ("status", ctypes.c_int32),
                ("reserved", ctypes.c_int32)]


class bte_instance(ctypes.Structure):
    _fields_ = [("E_dc", ctypes.c_double), ("E_w", ctypes.c_double),
                ("omega", ctypes.c_double), ("B", ctypes.c_double),
                ("mu", ctypes.c_double), ("n_y", ctypes.c_int32),
                ("reserved", ctypes.c_int32)]


class bte_batch_config(ctypes.Structure):
    _fields_ = [("n_x", ctypes.c_int32), ("precision", ctypes.c_int32),
                ("phiy_min", ctypes.c_double), ("phiy_max", ctypes.c_double),
                ("dt", ctypes.c_double), ("alpha", ctypes.c_double),
                ("tol", ctypes.c_double), ("min_periods", ctypes.c_int32),
                ("max_periods", ctypes.c_int32), ("confirm", ctypes.c_int32),
                ("reserved", ctypes.c_int32)]


class bte_batch_tuning(ctypes.Structure):
    _fields_ = [("kernel", ctypes.c_int32), ("rows_per_wave", ctypes.c_int32),
                ("waves_per_group", ctypes.c_int32), ("groups", ctypes.c_int32),
                ("schedule", ctypes.c_int32)]


class bte_result(ctypes.Structure):
    _fields_ = [("absorption", ctypes.c_double), ("v_avg", ctypes.c_double),
                ("dA", ctypes.c_double), ("steps", ctypes.c_int64),
                ("periods", ctypes.c_int32), ("converged", ctypes.c_int32),
                ("status", ctypes.c_int32), ("reserved", ctypes.c_int32)]


class BteError(RuntimeError):
    def __init__(self, status: int, func: str, msg: str):
        super().__init__(f"{func}: {STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"HIP library {LIB_PATH} is not built; run "
                          "`python -m paper_1401_6047_amd.build`")
    # torch provides device memory and streams: its HIP runtime has to be in
    # the process before the library binds to one, so that both share it
    # (loaded the other way round, the library's runtime saw no device)
    import torch  # noqa: F401
    lib = ctypes.CDLL(LIB_PATH)
    P = ctypes.POINTER
    vp, dp = ctypes.c_void_p, P(ctypes.c_double)
    sig = {
        "bte_workspace_bytes": ([P(bte_grid), P(bte_params), P(ctypes.c_size_t)], ctypes.c_int),
        "bte_create": ([P(bte_grid), P(bte_params), vp, ctypes.c_size_t, vp, P(vp)], ctypes.c_int),
        "bte_step": ([vp, ctypes.c_int64], ctypes.c_int),
        "bte_set_window": ([vp, ctypes.c_int64, ctypes.c_int64], ctypes.c_int),
        "bte_observables": ([vp, P(bte_obs)], ctypes.c_int),
        "bte_get_state": ([vp, dp, dp, dp, dp], ctypes.c_int),
        "bte_set_state": ([vp, dp, dp, dp, dp, ctypes.c_int64], ctypes.c_int),
        "bte_set_tuning": ([vp, P(bte_tuning)], ctypes.c_int),
        "bte_get_tuning": ([vp, P(bte_tuning)], ctypes.c_int),
        "bte_tune": ([P(bte_grid), P(bte_params), vp, ctypes.c_size_t, vp, ctypes.c_int32,
                      ctypes.c_double, P(bte_tuning), dp], ctypes.c_int),
        "bte_reconstruct": ([vp, ctypes.c_int32, vp], ctypes.c_int),
        "bte_reconstruct_coeffs": ([vp, vp, ctypes.c_int32, ctypes.c_int32, ctypes.c_int64,
                                    ctypes.c_int32, vp, vp], ctypes.c_int),
        "bte_batch_workspace_bytes": ([P(bte_batch_config), ctypes.c_int32, P(bte_instance),
                                       P(bte_batch_tuning), P(ctypes.c_size_t)], ctypes.c_int),
        "bte_batch_create": ([P(bte_batch_config), ctypes.c_int32, P(bte_instance),
                              P(bte_batch_tuning), vp, ctypes.c_size_t, vp, P(vp)], ctypes.c_int),
        "bte_batch_set_warm_start": ([vp, vp], ctypes.c_int),
        "bte_batch_set_state_output": ([vp, vp], ctypes.c_int),
        "bte_batch_run": ([vp], ctypes.c_int),
        "bte_batch_advance": ([vp, ctypes.c_int32, P(ctypes.c_int32)], ctypes.c_int),
        "bte_batch_results": ([vp, P(bte_result)], ctypes.c_int),
        "bte_batch_get_tuning": ([vp, P(bte_batch_tuning)], ctypes.c_int),
        "bte_batch_destroy": ([vp], None),
        "bte_batch_tune": ([P(bte_batch_config), ctypes.c_int32, P(bte_instance), vp, ctypes.c_int32,
                            P(bte_batch_tuning), dp], ctypes.c_int),
        "bte_state_observables_bytes": ([ctypes.c_int32, P(ctypes.c_size_t)], ctypes.c_int),
        "bte_state_observables": ([vp, vp, ctypes.c_int32, ctypes.c_int32, ctypes.c_int64,
                                   ctypes.c_double, ctypes.c_double, ctypes.c_double, vp,
                                   ctypes.c_size_t, vp, vp], ctypes.c_int),
        "bte_state_observables_noalloc": ([vp, vp, ctypes.c_int32, ctypes.c_int32, ctypes.c_int64,
                                           ctypes.c_double, ctypes.c_double, ctypes.c_double, vp,
                                           vp], ctypes.c_int),
        "bte_run_periods": ([vp, ctypes.c_double, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                             P(bte_result)], ctypes.c_int),
        "bte_stream_copy": ([vp, vp, ctypes.c_size_t, vp], ctypes.c_int),
        "bte_destroy": ([vp], None),
        "bte_last_error": ([], ctypes.c_char_p),
        "bte_version": ([], ctypes.c_char_p),
    }
    for name, (args, res) in sig.items():
        f = getattr(lib, name)
        f.argtypes = args
        f.restype = res
    return lib


_lib = _load()


def header_functions(path: str = HEADER_PATH) -> list[str]:
    """Names of the functions declared in include/bte.h."""
    text = open(path).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(bte_[a-z_0-9]+)\s*\(", text)))


def lib():
    return _lib


def _check(rc: int, func: str):
    if rc != BTE_OK:
        raise BteError(rc, func, _lib.bte_last_error().decode())


def _dptr(a):
    if a is None:
        return None
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


# ---- the C entry points, same names --------------------------------------
def bte_workspace_bytes(grid: bte_grid, params: bte_params) -> int:
    n = ctypes.c_size_t(0)
    _check(_lib.bte_workspace_bytes(ctypes.byref(grid), ctypes.byref(params), ctypes.byref(n)),
           "bte_workspace_bytes")
    return int(n.value)


def bte_create(grid: bte_grid, params: bte_params, workspace_ptr: int, workspace_bytes: int,
               stream_ptr: int) -> int:
    h = ctypes.c_void_p(0)
    _check(_lib.bte_create(ctypes.byref(grid), ctypes.byref(params),
                           ctypes.c_void_p(workspace_ptr or None), workspace_bytes,
                           ctypes.c_void_p(stream_ptr or None), ctypes.byref(h)), "bte_create")
    return h.value


def bte_step(h: int, n_steps: int):
    _check(_lib.bte_step(ctypes.c_void_p(h), int(n_steps)), "bte_step")


def bte_set_window(h: int, lo: int, hi: int):
    _check(_lib.bte_set_window(ctypes.c_void_p(h), int(lo), int(hi)), "bte_set_window")


def bte_observables(h: int) -> bte_obs:
    o = bte_obs()
    _check(_lib.bte_observables(ctypes.c_void_p(h), ctypes.byref(o)), "bte_observables")
    return o


def bte_get_state(h: int, a_h=None, b_h=None, a_f=None, b_f=None):
    _check(_lib.bte_get_state(ctypes.c_void_p(h), _dptr(a_h), _dptr(b_h), _dptr(a_f), _dptr(b_f)),
           "bte_get_state")


def bte_set_state(h: int, a_h, b_h, a_f=None, b_f=None, step: int = 0):
    _check(_lib.bte_set_state(ctypes.c_void_p(h), _dptr(a_h), _dptr(b_h), _dptr(a_f), _dptr(b_f),
                              int(step)), "bte_set_state")


def bte_reconstruct(h: int, n_phix: int, out_ptr: int):
    _check(_lib.bte_reconstruct(ctypes.c_void_p(h), int(n_phix), ctypes.c_void_p(out_ptr or None)),
           "bte_reconstruct")


def bte_reconstruct_coeffs(a_ptr: int, b_ptr: int, n_x: int, n_y: int, ld: int, n_phix: int,
                           out_ptr: int, stream_ptr: int):
    _check(_lib.bte_reconstruct_coeffs(ctypes.c_void_p(a_ptr or None), ctypes.c_void_p(b_ptr or None),
                                       int(n_x), int(n_y), int(ld), int(n_phix),
                                       ctypes.c_void_p(out_ptr or None),
                                       ctypes.c_void_p(stream_ptr or None)),
           "bte_reconstruct_coeffs")


def reconstruct(a, b, n_phix: int, out=None, stream=None):
    """f(phi_x_j, phi_y_m) from FP64 CUDA coefficient tensors a, b of shape
    (N_x, N_y) (rows may be strided; elements contiguous) on the uniform
    phi_x grid x_j = -pi + 2 pi j / n_phix.  Returns (n_phix, N_y) float64."""
    import torch
    for t in (a, b):
        if t.dtype != torch.float64 or not t.is_cuda or t.dim() != 2 or t.stride(1) != 1:
            raise ValueError("a and b must be 2-D float64 CUDA tensors with contiguous rows")
    if a.shape != b.shape or a.stride(0) != b.stride(0):
        raise ValueError("a and b must have the same shape and row stride")
    nx, ny = a.shape
    if out is None:
        out = torch.empty((n_phix, ny), dtype=torch.float64, device=a.device)
    elif (out.dtype != torch.float64 or tuple(out.shape) != (n_phix, ny) or
          not out.is_contiguous()):
        raise ValueError("out must be a contiguous float64 tensor of shape (n_phix, N_y)")
    st = stream if stream is not None else torch.cuda.current_stream(a.device)
    bte_reconstruct_coeffs(a.data_ptr(), b.data_ptr(), nx, ny, a.stride(0), n_phix,
                           out.data_ptr(), st.cuda_stream)
    return out


def bte_set_tuning(h: int, t: bte_tuning):
    _check(_lib.bte_set_tuning(ctypes.c_void_p(h), ctypes.byref(t)), "bte_set_tuning")


def bte_get_tuning(h: int) -> bte_tuning:
    t = bte_tuning()
    _check(_lib.bte_get_tuning(ctypes.c_void_p(h), ctypes.byref(t)), "bte_get_tuning")
    return t


def bte_tune(grid: bte_grid, params: bte_params, workspace_ptr: int, workspace_bytes: int,
             stream_ptr: int, kernel_form: int = -1, target_ms: float = 2.0):
    t = bte_tuning()
    us = ctypes.c_double(0.0)
    _check(_lib.bte_tune(ctypes.byref(grid), ctypes.byref(params),
                         ctypes.c_void_p(workspace_ptr or None), workspace_bytes,
                         ctypes.c_void_p(stream_ptr or None), int(kernel_form), float(target_ms),
                         ctypes.byref(t), ctypes.byref(us)), "bte_tune")
    return t, us.value


def _inst_array(instances):
    arr = (bte_instance * len(instances))()
    for i, w in enumerate(instances):
        arr[i] = bte_instance(float(w.E_dc), float(w.E_w), float(w.omega), float(w.B),
                              float(w.mu), int(w.ny), 0)
    return arr


def bte_batch_workspace_bytes(cfg: bte_batch_config, instances, tuning=None) -> int:
    arr = _inst_array(instances)
    n = ctypes.c_size_t(0)
    _check(_lib.bte_batch_workspace_bytes(ctypes.byref(cfg), len(arr), arr,
                                          ctypes.byref(tuning) if tuning else None,
                                          ctypes.byref(n)), "bte_batch_workspace_bytes")
    return int(n.value)


def bte_batch_create(cfg, instances, tuning, workspace_ptr, workspace_bytes, stream_ptr) -> int:
    arr = _inst_array(instances)
    h = ctypes.c_void_p(0)
    _check(_lib.bte_batch_create(ctypes.byref(cfg), len(arr), arr,
                                 ctypes.byref(tuning) if tuning else None,
                                 ctypes.c_void_p(workspace_ptr or None), workspace_bytes,
                                 ctypes.c_void_p(stream_ptr or None), ctypes.byref(h)),
           "bte_batch_create")
    return h.value


def bte_batch_set_warm_start(h: int, dev_ptr: int):
    _check(_lib.bte_batch_set_warm_start(ctypes.c_void_p(h), ctypes.c_void_p(dev_ptr or None)),
           "bte_batch_set_warm_start")


def bte_batch_set_state_output(h: int, dev_ptr: int):
    _check(_lib.bte_batch_set_state_output(ctypes.c_void_p(h), ctypes.c_void_p(dev_ptr or None)),
           "bte_batch_set_state_output")


def bte_batch_run(h: int):
    _check(_lib.bte_batch_run(ctypes.c_void_p(h)), "bte_batch_run")


def bte_batch_advance(h: int, max_replays: int) -> int:
    left = ctypes.c_int32(0)
    _check(_lib.bte_batch_advance(ctypes.c_void_p(h), int(max_replays), ctypes.byref(left)),
           "bte_batch_advance")
    return int(left.value)


def bte_batch_results(h: int, n: int):
    out = (bte_result * n)()
    _check(_lib.bte_batch_results(ctypes.c_void_p(h), out), "bte_batch_results")
    return out


def bte_batch_get_tuning(h: int) -> bte_batch_tuning:
    t = bte_batch_tuning()
    _check(_lib.bte_batch_get_tuning(ctypes.c_void_p(h), ctypes.byref(t)), "bte_batch_get_tuning")
    return t


def bte_run_periods(h: int, tol: float, min_periods: int, max_periods: int,
                    confirm: int) -> bte_result:
    r = bte_result()
    _check(_lib.bte_run_periods(ctypes.c_void_p(h), float(tol), int(min_periods),
                                int(max_periods), int(confirm), ctypes.byref(r)),
           "bte_run_periods")
    return r


def bte_state_observables_bytes(n_x: int) -> int:
    n = ctypes.c_size_t(0)
    _check(_lib.bte_state_observables_bytes(int(n_x), ctypes.byref(n)),
           "bte_state_observables_bytes")
    return int(n.value)


def bte_state_observables(a_ptr, b_ptr, n_x, n_y, ld, phiy_min, phiy_max, alpha, ws_ptr,
                          ws_bytes, stream_ptr, out_ptr):
    _check(_lib.bte_state_observables(ctypes.c_void_p(a_ptr or None), ctypes.c_void_p(b_ptr or None),
                                      int(n_x), int(n_y), int(ld), float(phiy_min),
                                      float(phiy_max), float(alpha), ctypes.c_void_p(ws_ptr or None),
                                      int(ws_bytes), ctypes.c_void_p(stream_ptr or None),
                                      ctypes.c_void_p(out_ptr or None)), "bte_state_observables")


def bte_stream_copy(src_ptr, dst_ptr, nbytes, stream_ptr=0):
    _check(_lib.bte_stream_copy(ctypes.c_void_p(src_ptr or None), ctypes.c_void_p(dst_ptr or None),
                                int(nbytes), ctypes.c_void_p(stream_ptr or None)),
           "bte_stream_copy")


STATE_OBS_NOALLOC_MAX_NX = 16384   # BTE_STATE_OBS_NOALLOC_MAX_NX of include/bte.h


def bte_state_observables_noalloc(a_ptr, b_ptr, n_x, n_y, ld, phiy_min, phiy_max, alpha,
                                  stream_ptr, out_ptr):
    _check(_lib.bte_state_observables_noalloc(
        ctypes.c_void_p(a_ptr or None), ctypes.c_void_p(b_ptr or None), int(n_x), int(n_y),
        int(ld), float(phiy_min), float(phiy_max), float(alpha),
        ctypes.c_void_p(stream_ptr or None), ctypes.c_void_p(out_ptr or None)),
        "bte_state_observables_noalloc")


def state_observables(a, b, phiy_min, phiy_max, alpha=1.0, workspace=None, stream=None):
    """(norm, v_dr, edge_mass, top_harm_mass) of FP64 CUDA coefficient tensors
    a, b of shape (N_x, N_y) (rows may be strided; elements contiguous), as a
    float64 CUDA tensor of 4.  `workspace`: a uint8 CUDA tensor of at least
    bte_state_observables_bytes(N_x) + 256 bytes, or None to allocate one."""
    import torch
    for t in (a, b):
        if t.dtype != torch.float64 or not t.is_cuda or t.dim() != 2 or t.stride(1) != 1:
            raise ValueError("a and b must be 2-D float64 CUDA tensors with contiguous rows")
    if a.shape != b.shape or a.stride(0) != b.stride(0):
        raise ValueError("a and b must have the same shape and row stride")
    nx, ny = a.shape
    need = bte_state_observables_bytes(nx)
    if workspace is None:
        workspace = torch.empty(need + 256, dtype=torch.uint8, device=a.device)
    ptr = (workspace.data_ptr() + 255) // 256 * 256
    if ptr + need > workspace.data_ptr() + workspace.numel():
        raise ValueError("workspace too small")
    out = torch.empty(4, dtype=torch.float64, device=a.device)
    st = stream if stream is not None else torch.cuda.current_stream(a.device)
    bte_state_observables(a.data_ptr(), b.data_ptr(), nx, ny, a.stride(0), phiy_min, phiy_max,
                          alpha, ptr, need, st.cuda_stream, out.data_ptr())
    return out


def bte_batch_destroy(h: int):
    _lib.bte_batch_destroy(ctypes.c_void_p(h))


def bte_destroy(h: int):
    _lib.bte_destroy(ctypes.c_void_p(h))


def bte_last_error() -> str:
    return _lib.bte_last_error().decode()


def bte_version() -> str:
    return _lib.bte_version().decode()


# ---- convenience wrapper ---------------------------------------------------
def make_grid(n_x, n_y, phiy_min, phiy_max) -> bte_grid:
    return bte_grid(int(n_x), int(n_y), float(phiy_min), float(phiy_max))


def make_params(E_dc, E_w, omega, B, mu, dt, alpha=1.0, tau=1.0, precision=BTE_FP64) -> bte_params:
    return bte_params(float(E_dc), float(E_w), float(omega), float(B), float(mu), float(alpha),
                      float(tau), float(dt), int(precision), 0)


class Solver:
    """One solver instance on the current torch device and stream.

    The workspace is a torch uint8 tensor owned by this object; torch's
    current stream is the stream every launch is queued on."""

    def __init__(self, grid: bte_grid, params: bte_params, device="cuda", stream=None):
        import torch
        self.grid, self.params = grid, params
        nbytes = bte_workspace_bytes(grid, params)
        self.workspace = torch.empty(nbytes + 256, dtype=torch.uint8, device=device)
        base = self.workspace.data_ptr()
        ptr = (base + 255) // 256 * 256
        self.stream = stream if stream is not None else torch.cuda.current_stream(device)
        self.handle = bte_create(grid, params, ptr, nbytes, self.stream.cuda_stream)

    @classmethod
    def from_workload(cls, w, precision=BTE_FP64, **kw):
        return cls(make_grid(w.nx, w.ny, w.phiy_min, w.phiy_max),
                   make_params(w.E_dc, w.E_w, w.omega, w.B, w.mu, w.dt, alpha=w.alpha,
                               precision=precision), **kw)

    def step(self, n: int):
        bte_step(self.handle, n)

    def set_window(self, lo: int, hi: int):
        bte_set_window(self.handle, lo, hi)

    def observables(self) -> bte_obs:
        return bte_observables(self.handle)

    def state(self):
        shape = (self.grid.n_x, self.grid.n_y)
        arrs = [np.zeros(shape) for _ in range(4)]
        bte_get_state(self.handle, *arrs)
        return tuple(arrs)

    def set_state(self, a_h, b_h, a_f=None, b_f=None, step=0):
        c = lambda x: None if x is None else np.ascontiguousarray(x, dtype=np.float64)
        bte_set_state(self.handle, c(a_h), c(b_h), c(a_f), c(b_f), step)

    def autotune(self, kernel_form: int = -1, target_ms: float = 2.0):
        """Pick the launch shape by measurement on a scratch copy of this
        solver's grid (a separate workspace; this solver's state is untouched)
        and apply it.  Returns (tuning, microseconds per step)."""
        import torch
        nbytes = bte_workspace_bytes(self.grid, self.params)
        scratch = torch.empty(nbytes + 256, dtype=torch.uint8, device=self.workspace.device)
        ptr = (scratch.data_ptr() + 255) // 256 * 256
        t, us = bte_tune(self.grid, self.params, ptr, nbytes, self.stream.cuda_stream,
                         kernel_form, target_ms)
        del scratch
        bte_set_tuning(self.handle, t)
        return t, us

    def tuning(self) -> bte_tuning:
        return bte_get_tuning(self.handle)

    def run_periods(self, tol=1e-6, min_periods=2, max_periods=400, confirm=1):
        """bte_run_periods: whole ac periods from the current step until the
        per-period absorption changes by less than `tol` on `confirm`
        consecutive periods (the batched sweep's criterion).  Returns a dict
        shaped like the entries of Batch.results()."""
        x = bte_run_periods(self.handle, tol, min_periods, max_periods, confirm)
        return dict(absorption=x.absorption, v_avg=x.v_avg, dA=x.dA, steps=x.steps,
                    periods=x.periods, converged=x.converged, status=x.status)

    def reconstruct(self, n_phix: int, out=None):
        """f(phi_x, phi_y) of the current whole-grid state on x_j = -pi +
        2 pi j / n_phix: a (n_phix, N_y) float64 tensor on this solver's
        device, filled on its stream."""
        import torch
        ny = self.grid.n_y
        if out is None:
            out = torch.empty((n_phix, ny), dtype=torch.float64, device=self.workspace.device)
        elif (out.dtype != torch.float64 or tuple(out.shape) != (n_phix, ny) or
              not out.is_contiguous()):
            raise ValueError("out must be a contiguous float64 tensor of shape (n_phix, N_y)")
        bte_reconstruct(self.handle, n_phix, out.data_ptr())
        return out

    def set_tuning(self, kernel=None, rows_per_wave=None, waves_per_block=None, graph_steps=None):
        t = self.tuning()
        if kernel is not None:
            t.kernel = kernel
        if rows_per_wave is not None:
            t.rows_per_wave = rows_per_wave
        if waves_per_block is not None:
            t.waves_per_block = waves_per_block
        if graph_steps is not None:
            t.graph_steps = graph_steps
        bte_set_tuning(self.handle, t)

    def close(self):
        if getattr(self, "handle", None):
            bte_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def make_batch_config(n_x, phiy_min, phiy_max, dt, precision=BTE_FP64, alpha=1.0, tol=1e-6,
                      min_periods=2, max_periods=200, confirm=1) -> bte_batch_config:
    return bte_batch_config(int(n_x), int(precision), float(phiy_min), float(phiy_max),
                            float(dt), float(alpha), float(tol), int(min_periods),
                            int(max_periods), int(confirm), 0)


def bte_batch_tune(cfg: bte_batch_config, instances, stream_ptr=0, use_cache=True):
    """(tuning, sample cell-steps/s) from the library's sweep autotuner."""
    arr = _inst_array(instances)
    t = bte_batch_tuning()
    rate = ctypes.c_double(0.0)
    _check(_lib.bte_batch_tune(ctypes.byref(cfg), len(arr), arr, ctypes.c_void_p(stream_ptr or None),
                               1 if use_cache else 0, ctypes.byref(t), ctypes.byref(rate)),
           "bte_batch_tune")
    return t, rate.value


def tuning_cache_key(cfg: bte_batch_config, instances) -> str:
    """Key of a batch tuning: harmonics, precision, the batch-size class (the
    smallest power of two at or above min(n, 4096)) and the set of N_y
    values, as the library's own cache keys it."""
    nys = sorted({int(w.ny) for w in instances})
    cls = 1
    while cls < min(len(instances), 4096):
        cls *= 2
    return f"nx{cfg.n_x}-p{cfg.precision}-n{cls}-ny" + ",".join(str(v) for v in nys)


class Batch:
    """A batched sweep of independent instances (see bte_batch_* in bte.h).

    `instances` are objects with E_dc, E_w, omega, B, mu, ny (e.g. Workload).
    With `tuning=None`: the two-step kernel, 58 harmonics per wave, 4
    wavefronts per group, and the wide schedule unless its per-instance slots
    would pass 64 GiB.  `autotune=True` takes the tile from the library's
    sweep autotuner (bte_batch_tune: a sample of this batch timed per
    candidate shape); `tuning_cache` names a JSON file that keeps its results
    across processes, keyed by (N_x, precision, set of N_y values)."""

    def __init__(self, cfg: bte_batch_config, instances, tuning=None, waves_per_group=4,
                 groups=0, device="cuda", stream=None, autotune=False, schedule=None,
                 tuning_cache=None):
        import torch
        self.cfg = cfg
        self.instances = list(instances)
        self.n = len(self.instances)
        self.stream = stream if stream is not None else torch.cuda.current_stream(device)
        self.tune_us = None
        if schedule is None:
            # wide (one state slot per instance) unless the slots would pass
            # 64 GiB, the library's own default rule
            ny = max(w.ny for w in self.instances)
            elem = 4 if cfg.precision == BTE_FP32_BULK else 8
            slot = 8 * (cfg.n_x + 8) * (ny + 128) * elem
            schedule = BTE_BATCH_WIDE if slot * self.n <= 64 * 2 ** 30 else BTE_BATCH_PERSISTENT
        self.tune_rate = None
        if tuning is None and autotune and schedule == BTE_BATCH_WIDE:
            tuning = self._autotune(cfg, tuning_cache)
        if tuning is None:
            tuning = bte_batch_tuning(BTE_KERNEL_FUSED2, 58, waves_per_group, groups, schedule)
        self.tuning = tuning
        nbytes = bte_batch_workspace_bytes(cfg, self.instances, tuning)
        self.workspace = torch.empty(nbytes + 256, dtype=torch.uint8, device=device)
        ptr = (self.workspace.data_ptr() + 255) // 256 * 256
        self.handle = bte_batch_create(cfg, self.instances, tuning, ptr, nbytes,
                                       self.stream.cuda_stream)
        self._warm = None

    def _autotune(self, cfg, cache_path):
        import json
        key = tuning_cache_key(cfg, self.instances)
        table = {}
        if cache_path and os.path.exists(cache_path):
            with open(cache_path) as f:
                table = json.load(f)
        if key in table:
            e = table[key]
            self.tune_rate = e.get("cell_steps_per_s")
            return bte_batch_tuning(e["kernel"], e["rows_per_wave"], e["waves_per_group"], 0,
                                    BTE_BATCH_WIDE)
        t, rate = bte_batch_tune(cfg, self.instances, self.stream.cuda_stream)
        self.tune_rate = rate
        if cache_path:
            table[key] = {"kernel": t.kernel, "rows_per_wave": t.rows_per_wave,
                          "waves_per_group": t.waves_per_group, "cell_steps_per_s": rate}
            with open(cache_path, "w") as f:
                json.dump(table, f, indent=1, sort_keys=True)
        return t

    def set_warm_start(self, coeffs):
        """coeffs: a contiguous float32 CUDA tensor of shape (n, 64, 128), or None."""
        if coeffs is None:
            self._warm = None
            bte_batch_set_warm_start(self.handle, 0)
            return
        assert coeffs.is_cuda and coeffs.dtype.is_floating_point and coeffs.is_contiguous()
        assert tuple(coeffs.shape) == (self.n, 64, 128)
        self._warm = coeffs
        bte_batch_set_warm_start(self.handle, coeffs.data_ptr())

    def set_state_output(self, out):
        """out: a contiguous float32 CUDA tensor of shape (n, 64, 128) that each
        run fills with the converged states (warm-start encoding), or None."""
        if out is None:
            self._out = None
            bte_batch_set_state_output(self.handle, 0)
            return
        assert out.is_cuda and out.dtype.is_floating_point and out.is_contiguous()
        assert tuple(out.shape) == (self.n, 64, 128)
        self._out = out
        bte_batch_set_state_output(self.handle, out.data_ptr())

    def run(self, wait=True, report_every=20.0, log=print):
        """Queue the sweep; with wait=True block until it finishes, printing the
        elapsed time every `report_every` seconds.  Returns wall seconds."""
        import time
        import torch
        t0 = time.perf_counter()
        if self.tuning.schedule == BTE_BATCH_WIDE:
            # the host drives the passes; advance in slices so that progress
            # can be reported
            last = t0
            left = bte_batch_advance(self.handle, 1)
            while left > 0:
                left = bte_batch_advance(self.handle, 16)
                now = time.perf_counter()
                if left and log and now - last >= report_every:
                    log(f"  batch of {self.n} instances: {left} running, {now - t0:.0f} s",
                        flush=True)
                    last = now
            return time.perf_counter() - t0
        done = torch.cuda.Event()
        bte_batch_run(self.handle)
        done.record(self.stream)
        if not wait:
            return 0.0
        last = t0
        while not done.query():
            time.sleep(0.05)
            now = time.perf_counter()
            if log and now - last >= report_every:
                log(f"  batch of {self.n} instances running: {now - t0:.0f} s", flush=True)
                last = now
        return time.perf_counter() - t0

    def results(self):
        r = bte_batch_results(self.handle, self.n)
        return [dict(absorption=x.absorption, v_avg=x.v_avg, dA=x.dA, steps=x.steps,
                     periods=x.periods, converged=x.converged, status=x.status) for x in r]

    def get_tuning(self) -> bte_batch_tuning:
        return bte_batch_get_tuning(self.handle)

    def close(self):
        if getattr(self, "handle", None):
            bte_batch_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
