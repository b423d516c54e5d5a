"""Thin Python binding of libgfors (include/gfors.h).

Argument marshalling only: every step of the method runs in the HIP library.
PyTorch supplies the device workspace (one uint8 tensor) and the HIP stream.
If the shared library is not built this module raises; there is no fallback.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libgfors.so")

GFORS_OK = 0
_ERRS = {-1: "GFORS_E_ARG", -2: "GFORS_E_NONINT", -3: "GFORS_E_OOM", -4: "GFORS_E_HIP",
         -5: "GFORS_E_STATE", -6: "GFORS_E_INFEAS_ROW"}

c_i32, c_i64, c_u64, c_dbl, c_vp = ctypes.c_int32, ctypes.c_int64, ctypes.c_uint64, ctypes.c_double, ctypes.c_void_p


class gfors_csr(ctypes.Structure):
    _fields_ = [("nrows", c_i64), ("ncols", c_i64), ("row_ptr", c_vp), ("col_idx", c_vp), ("val", c_vp)]


class gfors_params(ctypes.Structure):
    _fields_ = [("sigma", c_dbl), ("tau1", c_dbl), ("tau2", c_dbl),
                ("rho_min", c_dbl), ("rho_max", c_dbl), ("rho_T", c_dbl), ("rho_p", c_dbl),
                ("rho_delta", c_dbl), ("k_int", c_i32), ("K_max", c_i32), ("power_iters", c_i32),
                ("hist_cap", c_i32), ("autotune", c_i32), ("x0", c_dbl), ("seed", c_u64),
                ("eval_mfma", c_i32), ("repair_row0", c_i64), ("lu_wide_rows", c_i32),
                ("lu_lds", c_i32)]


EXPORTS = [
    "gfors_default_params", "gfors_workspace_bytes", "gfors_create_problem", "gfors_sample_eval_ex",
    "gfors_destroy_problem", "gfors_last_error", "gfors_pdhg_steps", "gfors_sample_eval",
    "gfors_final_round", "gfors_run_rounds", "gfors_best", "gfors_get_residuals",
    "gfors_get_history", "gfors_get_state", "gfors_set_state", "gfors_get_candidates",
    "gfors_get_scales", "gfors_get_dims", "gfors_kernel_times", "gfors_reset",
    "gfors_get_launch_cfg", "gfors_set_launch_cfg", "gfors_autotune",
    "gfors_gnn_workspace_bytes", "gfors_gnn_create", "gfors_gnn_destroy", "gfors_gnn_act_bytes",
    "gfors_gnn_forward", "gfors_gnn_grad", "gfors_gnn_adam", "gfors_gnn_train_step",
    "gfors_gnn_get_params", "gfors_gnn_set_params", "gfors_gnn_get_grad", "gfors_gnn_set_grad",
    "gfors_tu_create", "gfors_tu_dims", "gfors_tu_export", "gfors_tu_recover", "gfors_tu_destroy",
    "gfors_tu_export_q", "gfors_sample_eval_assign3d",
    "gfors_tu_last_error", "gfors_mono_rows", "gfors_mono_repair", "gfors_mono_last_error",
    "gfors_philox_throughput", "gfors_eval_planes", "gfors_create_problem_static",
    "gfors_tu_create_ex", "gfors_tu_factor_info", "gfors_workspace_bytes_tu", "gfors_create_problem_tu",
    "gfors_read_throughput",
]

GFORS_TU_FACTORED = 1

KERNEL_NAMES = ["dual", "primal", "sample", "eval_cover", "eval_general", "eval_quad",
                "reduce_cand", "argmin_update", "extract_best"]

_lib = None


def load_library(path: str = LIB_PATH) -> ctypes.CDLL:
    """Load libgfors.so and declare its signatures.  Raises if it is missing."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is not built; run __graft_entry__.build() first")
    L = ctypes.CDLL(path)
    P = ctypes.POINTER
    L.gfors_default_params.argtypes = [P(gfors_params)]
    L.gfors_default_params.restype = None
    L.gfors_workspace_bytes.argtypes = [c_i64, c_i64, c_i64, c_i64, c_i64, c_i64, c_i32,
                                        P(gfors_params), P(ctypes.c_size_t)]
    L.gfors_create_problem.argtypes = [P(gfors_csr), c_vp, P(gfors_csr), c_vp, P(gfors_csr), c_vp,
                                       c_i64, c_i32, c_vp, P(gfors_params), c_vp, ctypes.c_size_t,
                                       c_vp, P(c_vp)]
    L.gfors_create_problem_static.argtypes = [P(gfors_csr), c_vp, P(gfors_csr), c_vp, P(gfors_csr),
                                              c_vp, c_i64, c_i32, c_vp, P(gfors_params), c_vp, P(c_vp)]
    L.gfors_destroy_problem.argtypes = [c_vp]
    L.gfors_destroy_problem.restype = None
    L.gfors_last_error.argtypes = []
    L.gfors_last_error.restype = ctypes.c_char_p
    L.gfors_pdhg_steps.argtypes = [c_vp, c_i32, c_i32]
    L.gfors_sample_eval.argtypes = [c_vp, c_i32, c_vp, c_vp, c_vp]
    L.gfors_final_round.argtypes = [c_vp]
    L.gfors_sample_eval_ex.argtypes = [c_vp, c_i32, c_vp, c_vp, c_vp, c_i32]
    L.gfors_run_rounds.argtypes = [c_vp, c_i32, c_i32, c_i32]
    L.gfors_sample_eval_assign3d.argtypes = [c_vp, c_i32, c_i32, c_i32, c_i32, c_vp, c_vp, c_vp, c_i32]
    L.gfors_best.argtypes = [c_vp, c_i32, P(c_i64), c_vp, P(c_i32), c_vp]
    L.gfors_get_residuals.argtypes = [c_vp, c_vp]
    L.gfors_get_history.argtypes = [c_vp, c_i32, c_vp, c_i32, P(c_i32)]
    L.gfors_get_state.argtypes = [c_vp, c_vp, c_vp, c_vp, c_vp, P(c_i64), P(c_i64), P(c_i64)]
    L.gfors_set_state.argtypes = [c_vp, c_vp, c_vp, c_vp, c_vp, c_i64, c_i64, c_i64]
    L.gfors_get_candidates.argtypes = [c_vp, c_vp, P(c_i32)]
    L.gfors_get_scales.argtypes = [c_vp] + [c_vp] * 9
    L.gfors_get_dims.argtypes = [c_vp, P(c_i64), P(c_i64), P(c_i64), P(c_i32)]
    L.gfors_kernel_times.argtypes = [c_vp, c_i32, c_i32, c_vp, c_vp]
    L.gfors_reset.argtypes = [c_vp]
    L.gfors_get_launch_cfg.argtypes = [c_vp, c_vp]
    L.gfors_eval_planes.argtypes = [c_vp, P(c_i32)]
    L.gfors_set_launch_cfg.argtypes = [c_vp, c_vp]
    L.gfors_autotune.argtypes = [c_vp]
    L.gfors_gnn_workspace_bytes.argtypes = [P(ctypes.c_size_t)]
    L.gfors_gnn_create.argtypes = [c_vp, c_vp, ctypes.c_size_t, c_vp, P(c_vp)]
    L.gfors_gnn_destroy.argtypes = [c_vp]
    L.gfors_gnn_destroy.restype = None
    L.gfors_gnn_act_bytes.argtypes = [c_vp, c_i32, P(ctypes.c_size_t)]
    L.gfors_gnn_forward.argtypes = [c_vp, c_vp, c_vp, c_vp, c_vp, ctypes.c_size_t, c_vp, c_vp]
    L.gfors_gnn_grad.argtypes = [c_vp, c_vp, c_vp, c_vp, c_vp, c_vp, ctypes.c_size_t, c_vp]
    L.gfors_gnn_adam.argtypes = [c_vp, ctypes.c_float]
    L.gfors_gnn_train_step.argtypes = [c_vp, c_vp, c_vp, c_vp, c_vp, c_vp, ctypes.c_size_t,
                                       ctypes.c_float, c_vp]
    for nm in ("gfors_gnn_get_params", "gfors_gnn_set_params", "gfors_gnn_get_grad", "gfors_gnn_set_grad"):
        getattr(L, nm).argtypes = [c_vp, c_vp]
    L.gfors_tu_create.argtypes = [P(gfors_csr), c_vp, P(gfors_csr), c_vp, P(gfors_csr), c_vp, c_i64,
                                  c_vp, P(c_vp)]
    L.gfors_tu_create_ex.argtypes = [P(gfors_csr), c_vp, P(gfors_csr), c_vp, P(gfors_csr), c_vp, c_i64,
                                     c_vp, c_i32, P(c_vp)]
    L.gfors_tu_factor_info.argtypes = [c_vp, c_vp]
    L.gfors_workspace_bytes_tu.argtypes = [c_vp, P(gfors_params), P(ctypes.c_size_t)]
    L.gfors_create_problem_tu.argtypes = [c_vp, P(gfors_params), c_vp, ctypes.c_size_t, c_vp, P(c_vp)]
    L.gfors_tu_dims.argtypes = [c_vp, c_vp]
    L.gfors_tu_export.argtypes = [c_vp] + [c_vp] * 10
    L.gfors_tu_export_q.argtypes = [c_vp, c_vp, c_vp, c_vp]
    L.gfors_tu_recover.argtypes = [c_vp, c_vp, c_vp]
    L.gfors_tu_destroy.argtypes = [c_vp]
    L.gfors_tu_destroy.restype = None
    L.gfors_tu_last_error.argtypes = []
    L.gfors_tu_last_error.restype = ctypes.c_char_p
    L.gfors_mono_rows.argtypes = [c_vp, c_vp, c_vp, c_vp, c_vp, ctypes.c_int64, c_vp]
    L.gfors_mono_repair.argtypes = [c_vp, c_vp, c_vp, ctypes.c_int64, c_vp]
    L.gfors_philox_throughput.argtypes = [c_vp, c_i64, c_vp, P(c_dbl)]
    L.gfors_read_throughput.argtypes = [c_vp, c_vp, c_i64, c_i32, c_vp, P(c_dbl)]
    L.gfors_mono_last_error.argtypes = []
    L.gfors_mono_last_error.restype = ctypes.c_char_p
    for name in EXPORTS:
        f = getattr(L, name)
        if name not in ("gfors_default_params", "gfors_destroy_problem", "gfors_last_error",
                        "gfors_gnn_destroy", "gfors_tu_destroy", "gfors_tu_last_error",
                        "gfors_mono_last_error"):
            f.restype = c_i32
    _lib = L
    return L


class GforsError(RuntimeError):
    pass


def _check(rc: int):
    if rc != GFORS_OK:
        msg = load_library().gfors_last_error().decode(errors="replace")
        raise GforsError(f"{_ERRS.get(rc, rc)}: {msg}")


def _ptr(a: Optional[np.ndarray]):
    return None if a is None else ctypes.c_void_p(a.ctypes.data)


def default_params(**overrides) -> gfors_params:
    p = gfors_params()
    load_library().gfors_default_params(ctypes.byref(p))
    for k, v in overrides.items():
        if not hasattr(p, k):
            raise KeyError(k)
        setattr(p, k, v)
    return p


def philox_throughput(calls: int = 2_000_000_000, device: str = "cuda:0") -> float:
    """Calls per second of the sampler's Philox4x32-10 generator alone on the
    device (the peak for the sampler's ALU roofline)."""
    import torch
    L = load_library()
    dev = torch.device(device)
    sink = torch.zeros(1, dtype=torch.int32, device=dev)
    stream = torch.cuda.current_stream(dev)
    out = c_dbl(0.0)
    _check(L.gfors_philox_throughput(ctypes.c_void_p(stream.cuda_stream), int(calls),
                                     ctypes.c_void_p(sink.data_ptr()), ctypes.byref(out)))
    return float(out.value)


def read_throughput(nbytes: int = 512 << 20, workgroups: int = 1024, device: str = "cuda:0") -> float:
    """Bytes per second of a bare streaming read of nbytes on the device with
    the given number of 256-lane workgroups (gfors_read_throughput)."""
    import torch
    L = load_library()
    dev = torch.device(device)
    buf = torch.ones(nbytes // 4, dtype=torch.int32, device=dev)
    sink = torch.zeros(1, dtype=torch.int32, device=dev)
    stream = torch.cuda.current_stream(dev)
    out = c_dbl(0.0)
    _check(L.gfors_read_throughput(ctypes.c_void_p(stream.cuda_stream), ctypes.c_void_p(buf.data_ptr()),
                                   int(buf.numel() * 4), int(workgroups), ctypes.c_void_p(sink.data_ptr()),
                                   ctypes.byref(out)))
    return float(out.value)


def _csr(M, keep: list):
    if M is None:
        return None
    rp = np.ascontiguousarray(M.row_ptr, dtype=np.int64)
    col = np.ascontiguousarray(M.col, dtype=np.int32)
    val = None if M.val is None else np.ascontiguousarray(M.val, dtype=np.int32)
    keep += [rp, col, val]
    s = gfors_csr(M.nrows, M.ncols, rp.ctypes.data, col.ctypes.data if col.size else None,
                  None if val is None else (val.ctypes.data if val.size else None))
    keep.append(s)
    return s


class Problem:
    """One GFORS problem bound to a device workspace and a HIP stream.

    ``bip`` is a paper_2510_27117_amd.instances.BIP (integer CSR data).
    ``static_ws=True`` creates it with gfors_create_problem_static: no device
    workspace is allocated, the library's static array on the device is used
    (one live problem per device, at most GFORS_STATIC_WS_BYTES)."""

    def __init__(self, bip, params: Optional[gfors_params] = None, device: str = "cuda:0",
                 stream=None, static_ws: bool = False, tu=None):
        import torch
        L = load_library()
        self.torch = torch
        self.params = params if params is not None else default_params()
        if tu is not None:
            self._init_tu(tu, device, stream)
            return
        self.n = int(bip.n)
        self.m1, self.m2 = int(bip.m1), int(bip.m2)
        self.T = int(bip.num_instances)
        self.device = torch.device(device)
        nnzA = 0 if bip.A is None else bip.A.nnz
        nnzB = 0 if bip.B is None else bip.B.nnz
        nnzQ = 0 if bip.Q is None else bip.Q.nnz
        nbytes = ctypes.c_size_t(0)
        _check(L.gfors_workspace_bytes(self.n, self.m1, self.m2, nnzA, nnzB, nnzQ, self.T,
                                       ctypes.byref(self.params), ctypes.byref(nbytes)))
        self.ws_bytes = int(nbytes.value)
        self.static_ws = bool(static_ws)
        self.ws = (None if self.static_ws
                   else torch.empty(self.ws_bytes, dtype=torch.uint8, device=self.device))
        # a dedicated stream: the legacy null stream cannot be captured into graphs
        self.stream = stream if stream is not None else torch.cuda.Stream(device=self.device)
        keep: list = []
        A = _csr(bip.A, keep)
        B = _csr(bip.B, keep)
        Q = _csr(bip.Q, keep)
        b = None if bip.b is None else np.ascontiguousarray(bip.b, dtype=np.int64)
        d = None if bip.d is None else np.ascontiguousarray(bip.d, dtype=np.int64)
        c = np.ascontiguousarray(bip.c, dtype=np.int64)
        off = None
        if self.T > 1:
            off = np.ascontiguousarray(bip.inst_offsets, dtype=np.int64).reshape(-1)
        self.inst_offsets = (np.asarray(bip.inst_offsets, dtype=np.int64) if bip.inst_offsets is not None
                             else np.array([[0, 0, 0], [self.n, self.m1, self.m2]], dtype=np.int64))
        h = ctypes.c_void_p()
        with torch.cuda.device(self.device):
            if self.static_ws:
                _check(L.gfors_create_problem_static(
                    ctypes.byref(A) if A else None, _ptr(b), ctypes.byref(B) if B else None, _ptr(d),
                    ctypes.byref(Q) if Q else None, _ptr(c), self.n, self.T, _ptr(off),
                    ctypes.byref(self.params), ctypes.c_void_p(self.stream.cuda_stream),
                    ctypes.byref(h)))
            else:
                _check(L.gfors_create_problem(
                    ctypes.byref(A) if A else None, _ptr(b), ctypes.byref(B) if B else None, _ptr(d),
                    ctypes.byref(Q) if Q else None, _ptr(c), self.n, self.T, _ptr(off),
                    ctypes.byref(self.params), ctypes.c_void_p(self.ws.data_ptr()),
                    ctypes.c_size_t(self.ws_bytes), ctypes.c_void_p(self.stream.cuda_stream),
                    ctypes.byref(h)))
        self.handle = h
        self.m = self.m1 + self.m2

    def _init_tu(self, tu, device, stream):
        """A problem in the factorised TU form (gfors_create_problem_tu) on the
        kept variables of a TUReformulation made with factored=True."""
        torch = self.torch
        L = load_library()
        self.tu = tu          # the handle must stay alive while the problem is created
        self.n, self.m1, self.m2 = tu.n_reduced, tu.m1, tu.m2
        self.T = 1
        self.device = torch.device(device)
        nbytes = ctypes.c_size_t(0)
        _check(L.gfors_workspace_bytes_tu(tu.handle, ctypes.byref(self.params), ctypes.byref(nbytes)))
        self.ws_bytes = int(nbytes.value)
        self.static_ws = False
        self.ws = torch.empty(self.ws_bytes, dtype=torch.uint8, device=self.device)
        self.stream = stream if stream is not None else torch.cuda.Stream(device=self.device)
        self.inst_offsets = np.array([[0, 0, 0], [self.n, self.m1, self.m2]], dtype=np.int64)
        h = ctypes.c_void_p()
        with torch.cuda.device(self.device):
            _check(L.gfors_create_problem_tu(tu.handle, ctypes.byref(self.params),
                                             ctypes.c_void_p(self.ws.data_ptr()), ctypes.c_size_t(self.ws_bytes),
                                             ctypes.c_void_p(self.stream.cuda_stream), ctypes.byref(h)))
        self.handle = h
        self.m = self.m1 + self.m2

    # --------------------------------------------------------------- calls
    def _h(self):
        if not self.handle:
            raise GforsError("problem already destroyed")
        return self.handle

    def pdhg_steps(self, nsteps: int, want_residuals: bool = False):
        _check(load_library().gfors_pdhg_steps(self._h(), int(nsteps), 1 if want_residuals else 0))

    def sample_eval(self, K: int, p_override=None, outputs: bool = False, trigger: bool = True):
        """One sampling round of K candidates per instance.  p_override: a float32
        device tensor of length n (values in [0,1]).  With outputs=True returns
        device tensors (viol int32 [T,K], obj int64 [T,K])."""
        torch = self.torch
        pp = None
        if p_override is not None:
            assert p_override.dtype == torch.float32 and p_override.is_cuda and p_override.numel() == self.n
            pp = ctypes.c_void_p(p_override.contiguous().data_ptr())
            self._p_keep = p_override
        v = z = None
        if outputs:
            v = torch.empty((self.T, K), dtype=torch.int32, device=self.device)
            z = torch.empty((self.T, K), dtype=torch.int64, device=self.device)
        _check(load_library().gfors_sample_eval_ex(self._h(), int(K), pp,
                                                   None if v is None else ctypes.c_void_p(v.data_ptr()),
                                                   None if z is None else ctypes.c_void_p(z.data_ptr()),
                                                   0 if trigger else 1))
        if outputs:
            self.synchronize()
            return v, z
        return None

    def sample_eval_assign3d(self, n: int, K: int, gamma: int, L: int, p_override=None,
                             outputs: bool = False, trigger: bool = True):
        """One round of the customized 3D-assignment sampler (Algorithm 4)
        in place of the Bernoulli round; same outputs as sample_eval."""
        torch = self.torch
        pp = None
        if p_override is not None:
            assert p_override.dtype == torch.float32 and p_override.is_cuda and p_override.numel() == self.n
            pp = ctypes.c_void_p(p_override.contiguous().data_ptr())
            self._p_keep = p_override
        v = z = None
        if outputs:
            v = torch.empty((1, K), dtype=torch.int32, device=self.device)
            z = torch.empty((1, K), dtype=torch.int64, device=self.device)
        _check(load_library().gfors_sample_eval_assign3d(
            self._h(), int(n), int(K), int(gamma), int(L), pp,
            None if v is None else ctypes.c_void_p(v.data_ptr()),
            None if z is None else ctypes.c_void_p(z.data_ptr()), 0 if trigger else 1))
        if outputs:
            self.synchronize()
            return v, z
        return None

    def final_round(self):
        _check(load_library().gfors_final_round(self._h()))

    def run_rounds(self, nrounds: int, K: int, use_graph: bool = True):
        _check(load_library().gfors_run_rounds(self._h(), int(nrounds), int(K), 1 if use_graph else 0))

    def best(self, inst: int = 0, want_x: bool = True):
        z = c_i64(0)
        found = c_i32(0)
        info = np.zeros(4, dtype=np.int64)
        nv = int(self.inst_offsets[inst + 1, 0] - self.inst_offsets[inst, 0])
        x = np.zeros(nv, dtype=np.uint8) if want_x else None
        _check(load_library().gfors_best(self._h(), int(inst), ctypes.byref(z), _ptr(x),
                                         ctypes.byref(found), _ptr(info)))
        return {"z": int(z.value), "found": bool(found.value), "x": x, "k": int(info[0]),
                "round": int(info[1]), "l": int(info[2]), "ntrig": int(info[3])}

    def residuals(self) -> np.ndarray:
        out = np.zeros((self.T, 4), dtype=np.float64)
        _check(load_library().gfors_get_residuals(self._h(), _ptr(out)))
        return out

    def history(self, inst: int = 0, cap: int = 4096):
        h = np.zeros(cap, dtype=np.int64)
        cnt = c_i32(0)
        _check(load_library().gfors_get_history(self._h(), int(inst), _ptr(h), int(cap), ctypes.byref(cnt)))
        return h[: min(cap, cnt.value)]

    def get_state(self):
        x = np.zeros(self.n, dtype=np.float32)
        xp = np.zeros(self.n, dtype=np.float32)
        y = np.zeros(max(self.m, 1), dtype=np.float32)
        rho = np.zeros(self.T, dtype=np.float64)
        k, r, nt = c_i64(0), c_i64(0), c_i64(0)
        _check(load_library().gfors_get_state(self._h(), _ptr(x), _ptr(xp), _ptr(y), _ptr(rho),
                                              ctypes.byref(k), ctypes.byref(r), ctypes.byref(nt)))
        return {"x": x, "x_prev": xp, "y": y[: self.m], "rho": rho, "k": k.value,
                "round": r.value, "ntrig": nt.value}

    def set_state(self, x, x_prev, y, rho, k: int = 0, round: int = 0, ntrig: int = 0):
        x = np.ascontiguousarray(x, dtype=np.float32)
        xp = np.ascontiguousarray(x_prev, dtype=np.float32)
        yy = np.ascontiguousarray(y if self.m else np.zeros(1), dtype=np.float32)
        rr = np.ascontiguousarray(np.broadcast_to(np.asarray(rho, dtype=np.float64), (self.T,)))
        _check(load_library().gfors_set_state(self._h(), _ptr(x), _ptr(xp), _ptr(yy), _ptr(rr),
                                              int(k), int(round), int(ntrig)))

    def candidates(self) -> np.ndarray:
        K = c_i32(0)
        _check(load_library().gfors_get_candidates(self._h(), None, ctypes.byref(K)))
        out = np.zeros((self.n, K.value // 64), dtype=np.uint64)
        _check(load_library().gfors_get_candidates(self._h(), _ptr(out), ctypes.byref(K)))
        return out

    def scales(self) -> dict:
        T = self.T
        arrs = {k: np.zeros(T) for k in ["obj_scale", "K_norm", "Q_norm", "tau1", "tau2",
                                          "rho_min", "rho_max", "rho_delta"]}
        row = np.zeros(max(self.m, 1))
        _check(load_library().gfors_get_scales(self._h(), _ptr(row), *[_ptr(arrs[k]) for k in [
            "obj_scale", "K_norm", "Q_norm", "tau1", "tau2", "rho_min", "rho_max", "rho_delta"]]))
        arrs["row_scale"] = row[: self.m]
        return arrs

    def kernel_times(self, nsteps: int, K: int) -> dict:
        """HIP-event average duration (ms) and launch count of each kernel kind
        over nsteps PDHG steps + one sampling round (state advances)."""
        ms = np.zeros(len(KERNEL_NAMES), dtype=np.float64)
        cnt = np.zeros(len(KERNEL_NAMES), dtype=np.int32)
        _check(load_library().gfors_kernel_times(self._h(), int(nsteps), int(K), _ptr(ms), _ptr(cnt)))
        return {k: (float(ms[i]), int(cnt[i])) for i, k in enumerate(KERNEL_NAMES)}

    def eval_planes(self) -> int:
        """Digit planes of the matrix-core evaluation of the general rows (0: row by row)."""
        out = c_i32()
        _check(load_library().gfors_eval_planes(self._h(), ctypes.byref(out)))
        return int(out.value)

    def launch_cfg(self) -> dict:
        out = np.zeros(8, dtype=np.int32)
        _check(load_library().gfors_get_launch_cfg(self._h(), _ptr(out)))
        return {"lpr_dual": int(out[0]), "lpr_primal": int(out[1]),
                "slices_dual": int(out[2]), "slices_primal": int(out[3]),
                "sell_dual": int(out[4]), "sell_primal": int(out[5]),
                "bits_dual": int(out[6]), "bits_primal": int(out[7])}

    def set_launch_cfg(self, lpr_dual, lpr_primal, slices_dual=1, slices_primal=1,
                       sell_dual=0, sell_primal=0, bits_dual=0, bits_primal=0):
        cfg = np.array([lpr_dual, lpr_primal, slices_dual, slices_primal, sell_dual, sell_primal,
                        bits_dual, bits_primal], dtype=np.int32)
        _check(load_library().gfors_set_launch_cfg(self._h(), _ptr(cfg)))

    def autotune(self):
        """Re-time the SpMV launch shapes on the current iterate and keep the fastest."""
        _check(load_library().gfors_autotune(self._h()))

    def reset(self):
        """Restart from x0 with a cleared incumbent (Preprocess kept)."""
        _check(load_library().gfors_reset(self._h()))

    def synchronize(self):
        self.stream.synchronize()

    def close(self):
        if self.handle:
            self.synchronize()
            load_library().gfors_destroy_problem(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# Module-level names mirroring the C entry points.
def gfors_create_problem(bip, params=None, device="cuda:0", stream=None) -> Problem:
    return Problem(bip, params, device, stream)


def gfors_create_problem_static(bip, params=None, device="cuda:0", stream=None) -> Problem:
    return Problem(bip, params, device, stream, static_ws=True)


def gfors_pdhg_steps(P: Problem, nsteps: int, want_residuals: bool = False):
    P.pdhg_steps(nsteps, want_residuals)


def gfors_sample_eval(P: Problem, K: int, p_override=None, outputs: bool = False):
    return P.sample_eval(K, p_override, outputs)


def gfors_best(P: Problem, inst: int = 0):
    return P.best(inst)


# ---------------------------------------------------------------------------
# Learned sampling proposal
# ---------------------------------------------------------------------------
GNN_NUM_PARAMS = 50241
GNN_H, GNN_L = 64, 3


def gnn_param_shapes():
    """Flat parameter layout of include/gfors.h (order matters)."""
    shp = [("Uv", (4, GNN_H)), ("uv", (GNN_H,)), ("Uc", (4, GNN_H)), ("uc", (GNN_H,))]
    for l in range(GNN_L):
        shp += [(f"Wcc{l}", (GNN_H, GNN_H)), (f"Wcv{l}", (GNN_H, GNN_H)), (f"bc{l}", (GNN_H,)),
                (f"Wvv{l}", (GNN_H, GNN_H)), (f"Wvc{l}", (GNN_H, GNN_H)), (f"bv{l}", (GNN_H,))]
    shp += [("wo", (GNN_H,)), ("bo", (1,))]
    return shp


def gnn_init_params(seed: int = 0) -> np.ndarray:
    """Glorot-uniform weights, zero biases (seeded), as the flat FP32 vector."""
    rng = np.random.default_rng(seed)
    out = []
    for name, shp in gnn_param_shapes():
        if len(shp) == 2:
            lim = np.sqrt(6.0 / (shp[0] + shp[1]))
            out.append(rng.uniform(-lim, lim, size=shp).reshape(-1))
        elif name == "wo":
            lim = np.sqrt(6.0 / (GNN_H + 1))
            out.append(rng.uniform(-lim, lim, size=shp))
        else:
            out.append(np.zeros(shp))
    v = np.concatenate(out).astype(np.float32)
    assert v.size == GNN_NUM_PARAMS
    return v


class GNN:
    """A learned-proposal network living on the device."""

    def __init__(self, params: Optional[np.ndarray] = None, seed: int = 0, device: str = "cuda:0",
                 stream=None):
        import torch
        self.torch = torch
        L = load_library()
        nb = ctypes.c_size_t(0)
        _check(L.gfors_gnn_workspace_bytes(ctypes.byref(nb)))
        self.ws = torch.empty(int(nb.value), dtype=torch.uint8, device=device)
        self.stream = stream if stream is not None else torch.cuda.Stream(device=device)
        p = gnn_init_params(seed) if params is None else np.ascontiguousarray(params, dtype=np.float32)
        assert p.size == GNN_NUM_PARAMS
        h = ctypes.c_void_p()
        _check(L.gfors_gnn_create(_ptr(p), ctypes.c_void_p(self.ws.data_ptr()), nb.value,
                                  ctypes.c_void_p(self.stream.cuda_stream), ctypes.byref(h)))
        self.handle = h
        self._acts = {}

    def _act(self, prob: "Problem", training: bool):
        key = (id(prob), training)
        if key not in self._acts:
            nb = ctypes.c_size_t(0)
            _check(load_library().gfors_gnn_act_bytes(prob._h(), 1 if training else 0, ctypes.byref(nb)))
            self._acts[key] = self.torch.empty(int(nb.value), dtype=self.torch.uint8, device=prob.device)
        a = self._acts[key]
        return ctypes.c_void_p(a.data_ptr()), a.numel()

    @staticmethod
    def _dptr(t):
        return None if t is None else ctypes.c_void_p(t.data_ptr())

    def forward(self, prob: "Problem", x=None, y=None, with_logits: bool = False):
        """p = sigmoid(logit) (device float32 [n]); x, y: device float32 or None (current state)."""
        torch = self.torch
        p = torch.empty(prob.n, dtype=torch.float32, device=prob.device)
        lg = torch.empty(prob.n, dtype=torch.float32, device=prob.device) if with_logits else None
        a, nb = self._act(prob, False)
        _check(load_library().gfors_gnn_forward(self.handle, prob._h(), self._dptr(x), self._dptr(y),
                                                a, nb, self._dptr(p), self._dptr(lg)))
        return (p, lg) if with_logits else p

    def grad(self, prob, target, x=None, y=None) -> float:
        loss = ctypes.c_float(0)
        a, nb = self._act(prob, True)
        _check(load_library().gfors_gnn_grad(self.handle, prob._h(), self._dptr(x), self._dptr(y),
                                             self._dptr(target), a, nb, ctypes.byref(loss)))
        return float(loss.value)

    def train_step(self, prob, target, lr: float, x=None, y=None, want_loss: bool = True):
        loss = ctypes.c_float(0)
        a, nb = self._act(prob, True)
        _check(load_library().gfors_gnn_train_step(self.handle, prob._h(), self._dptr(x), self._dptr(y),
                                                   self._dptr(target), a, nb, ctypes.c_float(lr),
                                                   ctypes.byref(loss) if want_loss else None))
        return float(loss.value) if want_loss else None

    def adam(self, lr: float):
        _check(load_library().gfors_gnn_adam(self.handle, ctypes.c_float(lr)))

    def params(self) -> np.ndarray:
        v = np.zeros(GNN_NUM_PARAMS, dtype=np.float32)
        _check(load_library().gfors_gnn_get_params(self.handle, _ptr(v)))
        return v

    def set_params(self, v):
        v = np.ascontiguousarray(v, dtype=np.float32)
        _check(load_library().gfors_gnn_set_params(self.handle, _ptr(v)))

    def get_grad(self) -> np.ndarray:
        v = np.zeros(GNN_NUM_PARAMS, dtype=np.float32)
        _check(load_library().gfors_gnn_get_grad(self.handle, _ptr(v)))
        return v

    def set_grad(self, v):
        v = np.ascontiguousarray(v, dtype=np.float32)
        _check(load_library().gfors_gnn_set_grad(self.handle, _ptr(v)))

    def close(self):
        if self.handle:
            self.stream.synchronize()
            load_library().gfors_gnn_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ---------------------------------------------------------------------------
# TU reformulation (host-side C++ in the library)
# ---------------------------------------------------------------------------
class MonotoneRelaxation:
    """Monotone relaxation of set-partitioning equality rows (see
    gfors_mono_rows): ``model`` is the relaxed BIP, the relaxed rows appended
    to the inequality block with right-hand side 1; ``relaxed`` marks them
    among the original equality rows; ``repair(x)`` maps a relaxed point back
    (cheapest variable of each relaxed row kept).  The library decides and
    repairs; this class only moves rows between the two blocks."""

    def __init__(self, bip):
        from . import instances as _inst
        L = load_library()
        keep: list = []
        A = _csr(bip.A, keep)
        B = _csr(bip.B, keep)
        Q = _csr(bip.Q, keep)
        m2 = 0 if bip.B is None else bip.B.nrows
        d = None if bip.d is None else np.ascontiguousarray(bip.d, dtype=np.int64)
        c = np.ascontiguousarray(bip.c, dtype=np.int64)
        relax = np.zeros(max(m2, 1), dtype=np.uint8)
        rc = L.gfors_mono_rows(ctypes.byref(A) if A else None, ctypes.byref(B) if B else None,
                               _ptr(d), ctypes.byref(Q) if Q else None, _ptr(c), int(bip.n),
                               _ptr(relax))
        if rc != GFORS_OK:
            raise GforsError(f"{_ERRS.get(rc, rc)}: {L.gfors_mono_last_error().decode()}")
        self.relaxed = relax[:m2].astype(bool)
        self.source = bip
        self._c = c
        model = _inst.BIP(n=bip.n, c=bip.c.copy(), Q=bip.Q, name=bip.name + "_mono")
        if not self.relaxed.any():
            model.A, model.b, model.B, model.d = bip.A, bip.b, bip.B, bip.d
        else:
            rel = np.nonzero(self.relaxed)[0]
            kept = np.nonzero(~self.relaxed)[0]

            def take(M, rows):
                lens = np.array([M.row_ptr[r + 1] - M.row_ptr[r] for r in rows], dtype=np.int64)
                rp = np.concatenate([[0], np.cumsum(lens)]).astype(np.int64)
                idx = np.concatenate([np.arange(M.row_ptr[r], M.row_ptr[r + 1]) for r in rows]) \
                    if len(rows) else np.zeros(0, np.int64)
                col = np.asarray(M.col)[idx]
                val = None if M.val is None else np.asarray(M.val)[idx]
                return rp, col, val

            rpR, colR, valR = take(bip.B, rel)
            if bip.A is not None:
                rpA = np.asarray(bip.A.row_ptr, dtype=np.int64)
                colA = np.asarray(bip.A.col)
                valA = np.ones(bip.A.nnz, np.int32) if bip.A.val is None else np.asarray(bip.A.val)
                rp = np.concatenate([rpA, rpA[-1] + rpR[1:]])
                col = np.concatenate([colA, colR])
                val = np.concatenate([valA, np.ones(colR.size, np.int32) if valR is None else valR])
                b = np.concatenate([np.asarray(bip.b, np.int64), np.asarray(bip.d, np.int64)[rel]])
            else:
                rp, col = rpR, colR
                val = None if valR is None else valR
                b = np.asarray(bip.d, np.int64)[rel]
            model.A = _inst.CSR(len(rp) - 1, bip.n, rp, col.astype(np.int32),
                                None if val is None else val.astype(np.int32))
            model.b = b
            if kept.size:
                rpK, colK, valK = take(bip.B, kept)
                model.B = _inst.CSR(kept.size, bip.n, rpK, colK.astype(np.int32),
                                    None if valK is None else valK.astype(np.int32))
                model.d = np.asarray(bip.d, np.int64)[kept]
        self.model = model

    def repair(self, x) -> np.ndarray:
        xr = np.ascontiguousarray(np.asarray(x) != 0, dtype=np.uint8).copy()
        if not self.relaxed.any():
            return xr
        keep: list = []
        B = _csr(self.source.B, keep)
        relax = np.ascontiguousarray(self.relaxed, dtype=np.uint8)
        rc = load_library().gfors_mono_repair(ctypes.byref(B), _ptr(relax), _ptr(self._c),
                                              int(self.source.n), _ptr(xr))
        if rc != GFORS_OK:
            raise GforsError(f"{_ERRS.get(rc, rc)}: {load_library().gfors_mono_last_error().decode()}")
        return xr


class TUReformulation:
    """Eliminates one pivot variable per chosen equality row (gfors_tu_create:
    B_J totally unimodular, B_JI invertible; Q allowed).  ``model`` is the
    reformulated BIP (instances.BIP); ``constant`` is c'_0;
    ``recover(x_reduced)`` maps a reduced 0/1 point back.  With
    ``factored=True`` (gfors_tu_create_ex, GFORS_TU_FACTORED) no explicit
    model is formed (``model`` is None; ``b``, ``d``, ``c`` hold b', d', c');
    ``problem()`` makes the device problem that applies the LU of the pivot
    block at every step, ``info`` gives the factor and level counts."""

    def __init__(self, bip, pivots, factored: bool = False):
        from . import instances as _inst
        L = load_library()
        keep: list = []
        A = _csr(bip.A, keep)
        B = _csr(bip.B, keep)
        piv = np.ascontiguousarray(pivots, dtype=np.int64)
        assert bip.B is not None and piv.size == bip.B.nrows
        b = None if bip.b is None else np.ascontiguousarray(bip.b, dtype=np.int64)
        d = np.ascontiguousarray(bip.d, dtype=np.int64)
        c = np.ascontiguousarray(bip.c, dtype=np.int64)
        h = ctypes.c_void_p()
        Q = _csr(bip.Q, keep)
        rc = L.gfors_tu_create_ex(ctypes.byref(A) if A else None, _ptr(b), ctypes.byref(B), _ptr(d),
                                  ctypes.byref(Q) if Q else None, _ptr(c), int(bip.n), _ptr(piv),
                                  GFORS_TU_FACTORED if factored else 0, ctypes.byref(h))
        if rc != GFORS_OK:
            raise GforsError(f"{_ERRS.get(rc, rc)}: {L.gfors_tu_last_error().decode()}")
        self.handle = h
        self.factored = bool(factored)
        self.n_full = int(bip.n)
        dims = np.zeros(7, dtype=np.int64)
        L.gfors_tu_dims(h, _ptr(dims))
        n2, m1, m2, nA, nB, c0, nQ = (int(v) for v in dims)
        self.n_reduced, self.m1, self.m2 = n2, m1, m2
        self.constant = c0
        if factored:
            # no explicit rows: b', d', c' and the kept variables only
            bb, dd = np.zeros(max(m1, 1), np.int64), np.zeros(max(m2, 1), np.int64)
            cc, kept = np.zeros(n2, np.int64), np.zeros(n2, np.int64)
            L.gfors_tu_export(h, None, None, None, _ptr(bb), None, None, None, _ptr(dd), _ptr(cc), _ptr(kept))
            self.b, self.d, self.c, self.kept = bb[:m1], dd[:m2], cc, kept
            self.model = None
            info = np.zeros(10, dtype=np.int64)
            _check(L.gfors_tu_factor_info(h, _ptr(info)))
            self.info = dict(zip(("pivots", "nnz_L", "nnz_U", "levels_L", "levels_U", "levels_Ut",
                                  "levels_Lt", "nnz_BJ", "nnz_S", "nnz_reformulated_rows"),
                                 (int(v) for v in info)))
            return
        Arp, Aci, Aval, bb = (np.zeros(m1 + 1, np.int64), np.zeros(max(nA, 1), np.int32),
                              np.zeros(max(nA, 1), np.int32), np.zeros(max(m1, 1), np.int64))
        Brp, Bci, Bval, dd = (np.zeros(m2 + 1, np.int64), np.zeros(max(nB, 1), np.int32),
                              np.zeros(max(nB, 1), np.int32), np.zeros(max(m2, 1), np.int64))
        cc = np.zeros(n2, np.int64)
        kept = np.zeros(n2, np.int64)
        L.gfors_tu_export(h, _ptr(Arp), _ptr(Aci), _ptr(Aval), _ptr(bb), _ptr(Brp), _ptr(Bci),
                          _ptr(Bval), _ptr(dd), _ptr(cc), _ptr(kept))
        model = _inst.BIP(n=n2, c=cc, name=bip.name + "_tu")
        if m1:
            model.A = _inst.CSR(m1, n2, Arp, Aci[:nA], Aval[:nA])
            model.b = bb[:m1]
        if m2:
            model.B = _inst.CSR(m2, n2, Brp, Bci[:nB], Bval[:nB])
            model.d = dd[:m2]
        if nQ:
            Qrp, Qci, Qval = np.zeros(n2 + 1, np.int64), np.zeros(nQ, np.int32), np.zeros(nQ, np.int32)
            L.gfors_tu_export_q(h, _ptr(Qrp), _ptr(Qci), _ptr(Qval))
            model.Q = _inst.CSR(n2, n2, Qrp, Qci, Qval)
        self.model = model
        self.kept = kept

    def problem(self, params=None, device: str = "cuda:0", stream=None) -> "Problem":
        """The device problem of a factorised reformulation (gfors_create_problem_tu)."""
        assert self.factored, "problem() needs factored=True (else hand self.model to Problem)"
        return Problem(None, params, device=device, stream=stream, tu=self)

    def recover(self, x_reduced) -> np.ndarray:
        xr = np.ascontiguousarray(x_reduced, dtype=np.uint8)
        xf = np.zeros(self.n_full, dtype=np.uint8)
        rc = load_library().gfors_tu_recover(self.handle, _ptr(xr), _ptr(xf))
        if rc != GFORS_OK:
            raise GforsError(f"{_ERRS.get(rc, rc)}: {load_library().gfors_tu_last_error().decode()}")
        return xf

    def close(self):
        if self.handle:
            load_library().gfors_tu_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
