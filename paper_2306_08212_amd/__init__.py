"""MI355X corner-transfer (CTMRG) environments, reduced-cost move of Lan &
Evenbly (arXiv:2306.08212), behind the C-ABI library ``libctm.so``.

This module only marshals arguments: every step of a move runs in the HIP
kernels of ``libctm.so``.  PyTorch provides the device workspace and the
stream.  Importing works without a GPU; creating a solver needs one and
raises if the library is missing (nothing falls back to the CPU).
"""

from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass
from typing import Optional

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libctm.so")

CTM_OK, CTM_EINVAL, CTM_ENOMEM, CTM_EHIP, CTM_ENUMERIC, CTM_ENOTCONV = range(6)
STANDARD, REDUCED, REDUCED_ENV = 0, 1, 2
FP64, FP32, BF16 = 0, 1, 2
LEFT, UP, RIGHT, DOWN = 0, 1, 2, 3
PRECISIONS = {"fp64": FP64, "fp32": FP32, "bf16": BF16}
METHODS = {"standard": STANDARD, "reduced": REDUCED, "reduced_env": REDUCED_ENV}

EXPORTS = ["ctm_workspace_size", "ctm_init", "ctm_move", "ctm_iterate", "ctm_converge",
           "ctm_iterate_delta", "ctm_read_delta", "ctm_energy", "ctm_expect1", "ctm_row_correlation", "ctm_get_env", "ctm_set_env", "ctm_moves_done", "ctm_set_precision", "ctm_set_graphs",
           "ctm_profile", "ctm_profile_read", "ctm_destroy",
           "ctm_status_string", "ctm_kernel_gemm", "ctm_kernel_tsvd", "ctm_kernel_tsvd_workspace",
           "ctm_kernel_permute", "ctm_kernel_tsvd_static", "ctm_kernel_tsvd_static_max"]


class CtmConfig(ctypes.Structure):
    _fields_ = [("d", ctypes.c_int), ("D", ctypes.c_int), ("chi", ctypes.c_int),
                ("method", ctypes.c_int), ("precision", ctypes.c_int),
                ("boot_iters", ctypes.c_int), ("svd_cutoff", ctypes.c_double),
                ("stream", ctypes.c_void_p), ("workspace", ctypes.c_void_p),
                ("workspace_bytes", ctypes.c_size_t), ("chi_p", ctypes.c_int),
                ("chi_pp", ctypes.c_int)]


class CtmError(RuntimeError):
    def __init__(self, status: int, what: str):
        super().__init__(f"{what}: {status_string(status)} (status {status})")
        self.status = status


_lib = None


def load(path: str = LIB_PATH):
    """Load libctm.so (once) and declare its signatures."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise FileNotFoundError(
            f"{path} not found: build it with `python -m paper_2306_08212_amd.build`")
    # torch brings its own HIP runtime; load it first so that the library
    # binds to that one instead of starting a second runtime in the process
    import torch  # noqa: F401
    lib = ctypes.CDLL(path)
    P = ctypes.c_void_p
    I = ctypes.c_int
    D = ctypes.c_double
    lib.ctm_workspace_size.argtypes = [ctypes.POINTER(CtmConfig)]
    lib.ctm_workspace_size.restype = ctypes.c_size_t
    lib.ctm_init.argtypes = [ctypes.POINTER(CtmConfig), P, P, I, ctypes.POINTER(P)]
    lib.ctm_init.restype = I
    lib.ctm_move.argtypes = [P, I]
    lib.ctm_move.restype = I
    lib.ctm_iterate.argtypes = [P, I]
    lib.ctm_iterate.restype = I
    lib.ctm_converge.argtypes = [P, I, D, ctypes.POINTER(I), ctypes.POINTER(D)]
    lib.ctm_converge.restype = I
    lib.ctm_iterate_delta.argtypes = [P]
    lib.ctm_iterate_delta.restype = I
    lib.ctm_read_delta.argtypes = [P, ctypes.POINTER(D)]
    lib.ctm_read_delta.restype = I
    lib.ctm_energy.argtypes = [P, P, ctypes.POINTER(D), ctypes.POINTER(D)]
    lib.ctm_energy.restype = I
    lib.ctm_get_env.argtypes = [P, I, P, ctypes.c_size_t, ctypes.POINTER(I), ctypes.POINTER(I)]
    lib.ctm_get_env.restype = I
    lib.ctm_set_env.argtypes = [P, I, P, I, I]
    lib.ctm_set_env.restype = I
    lib.ctm_moves_done.argtypes = [P]
    lib.ctm_moves_done.restype = I
    lib.ctm_set_precision.argtypes = [P, I]
    lib.ctm_set_precision.restype = I
    lib.ctm_set_graphs.argtypes = [P, I]
    lib.ctm_set_graphs.restype = I
    lib.ctm_profile.argtypes = [P, I]
    lib.ctm_profile.restype = I
    lib.ctm_profile_read.argtypes = [P, I, ctypes.POINTER(ctypes.c_longlong),
                                     ctypes.POINTER(D), ctypes.POINTER(D), ctypes.POINTER(D)]
    lib.ctm_profile_read.restype = I
    lib.ctm_destroy.argtypes = [P]
    lib.ctm_destroy.restype = None
    lib.ctm_status_string.argtypes = [I]
    lib.ctm_status_string.restype = ctypes.c_char_p
    lib.ctm_kernel_gemm.argtypes = [I, I, I, I, D, P, ctypes.c_int64, I, P, ctypes.c_int64, I,
                                    D, P, ctypes.c_int64, P]
    lib.ctm_kernel_gemm.restype = I
    lib.ctm_kernel_tsvd.argtypes = [P, I, I, I, D, P, P, P, ctypes.c_size_t, P]
    lib.ctm_kernel_tsvd.restype = I
    lib.ctm_kernel_tsvd_workspace.argtypes = [I, I, I]
    lib.ctm_kernel_tsvd_workspace.restype = ctypes.c_size_t
    lib.ctm_expect1.argtypes = [P, P, ctypes.POINTER(D)]
    lib.ctm_expect1.restype = I
    lib.ctm_row_correlation.argtypes = [P, P, I, ctypes.POINTER(D)]
    lib.ctm_row_correlation.restype = I
    lib.ctm_kernel_tsvd_static.argtypes = [P, I, I, I, D, P, P, P]
    lib.ctm_kernel_tsvd_static.restype = I
    lib.ctm_kernel_tsvd_static_max.argtypes = []
    lib.ctm_kernel_tsvd_static_max.restype = ctypes.c_size_t
    lib.ctm_kernel_permute.argtypes = [I, P, I, ctypes.POINTER(ctypes.c_int64),
                                       ctypes.POINTER(I), I, P, D, P]
    lib.ctm_kernel_permute.restype = I
    _lib = lib
    return lib


def status_string(status: int) -> str:
    try:
        return load().ctm_status_string(int(status)).decode()
    except FileNotFoundError:
        return f"status {status}"


def _check(status: int, what: str, ok=(CTM_OK,)):
    if status not in ok:
        raise CtmError(status, what)
    return status


@dataclass
class Config:
    d: int = 2
    D: int = 2
    chi: int = 8
    method: int = REDUCED
    precision: int = FP64
    boot_iters: int = 0
    svd_cutoff: float = 1e-14
    chi_p: int = 0          # chi' of the sequential-order split (0 = chi)
    chi_pp: int = 0         # chi'' of the helper isometries (0 = chi)

    def to_c(self, stream=0, workspace=0, nbytes=0) -> CtmConfig:
        return CtmConfig(self.d, self.D, self.chi, self.method, self.precision,
                         self.boot_iters, self.svd_cutoff, stream or None,
                         workspace or None, nbytes, self.chi_p, self.chi_pp)


def workspace_size(cfg: Config) -> int:
    c = cfg.to_c()
    n = load().ctm_workspace_size(ctypes.byref(c))
    if n == 0:
        raise CtmError(CTM_EINVAL, "ctm_workspace_size")
    return int(n)


def _torch():
    import torch  # deferred: the CPU suite imports this module without a GPU
    return torch


class Solver:
    """One environment solve bound to one HIP stream.

    The workspace is a torch uint8 tensor on the current device; the solver
    keeps it alive until close().
    """

    def __init__(self, cfg: Config, A: np.ndarray, B: np.ndarray, stream=None,
                 workspace=None):
        torch = _torch()
        lib = load()
        self.cfg = cfg
        if stream is None:
            stream = torch.cuda.current_stream()
        self.stream = stream
        nbytes = workspace_size(cfg)
        if workspace is None:
            workspace = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
        self.workspace = workspace
        A = np.ascontiguousarray(A, dtype=np.float64)
        B = np.ascontiguousarray(B, dtype=np.float64)
        shape = (cfg.d, cfg.D, cfg.D, cfg.D, cfg.D)
        if A.shape != shape or B.shape != shape:
            raise ValueError(f"site tensors must have shape {shape}")
        c = cfg.to_c(stream.cuda_stream, workspace.data_ptr(), workspace.numel())
        h = ctypes.c_void_p()
        _check(lib.ctm_init(ctypes.byref(c), A.ctypes.data, B.ctypes.data, 0, ctypes.byref(h)),
               "ctm_init")
        self._h = h

    @property
    def handle(self):
        if self._h is None:
            raise RuntimeError("solver closed")
        return self._h

    def move(self, direction: int):
        _check(load().ctm_move(self.handle, direction), "ctm_move")

    def iterate(self, n: int = 1):
        _check(load().ctm_iterate(self.handle, n), "ctm_iterate")

    def converge(self, max_iters: int, tol: float):
        it = ctypes.c_int()
        dl = ctypes.c_double()
        st = load().ctm_converge(self.handle, max_iters, tol, ctypes.byref(it), ctypes.byref(dl))
        _check(st, "ctm_converge", ok=(CTM_OK, CTM_ENOTCONV))
        return it.value, dl.value, st == CTM_OK

    def iterate_delta(self):
        """Enqueue one iteration and its delta; returns at once."""
        _check(load().ctm_iterate_delta(self.handle), "ctm_iterate_delta")

    def read_delta(self) -> float:
        dl = ctypes.c_double()
        _check(load().ctm_read_delta(self.handle, ctypes.byref(dl)), "ctm_read_delta")
        return dl.value

    def energy(self, h2: Optional[np.ndarray] = None):
        e = ctypes.c_double()
        eb = (ctypes.c_double * 4)()
        hp = None
        if h2 is not None:
            h2 = np.ascontiguousarray(h2, dtype=np.float64)
            hp = h2.ctypes.data
        _check(load().ctm_energy(self.handle, hp, ctypes.byref(e), eb), "ctm_energy")
        return e.value, list(eb)

    def expect1(self, op: np.ndarray):
        """(<op>_a, <op>_b) of a d x d one-site operator (ctm_expect1)."""
        op = np.ascontiguousarray(op, dtype=np.float64)
        out = (ctypes.c_double * 2)()
        _check(load().ctm_expect1(self.handle, op.ctypes.data, out), "ctm_expect1")
        return list(out)

    def staggered_magnetisation(self) -> float:
        """|<S>_a - <S>_b| / 2 with S = sigma / 2; <S^y> = 0 for real tensors."""
        sx = np.array([[0.0, 0.5], [0.5, 0.0]])
        sz = np.array([[0.5, 0.0], [0.0, -0.5]])
        xa, xb = self.expect1(sx)
        za, zb = self.expect1(sz)
        return 0.5 * float(np.hypot(xa - xb, za - zb))

    def row_correlation(self, op: np.ndarray, L: int):
        """[C(1), ..., C(L)], C(x) = <op_0 op_x> - <op_0><op_x> along a row
        from an a-site (ctm_row_correlation)."""
        op = np.ascontiguousarray(op, dtype=np.float64)
        out = (ctypes.c_double * L)()
        _check(load().ctm_row_correlation(self.handle, op.ctypes.data, L, out),
               "ctm_row_correlation")
        return list(out)

    def get_env(self, e: int) -> np.ndarray:
        lib = load()
        p, q = ctypes.c_int(), ctypes.c_int()
        _check(lib.ctm_get_env(self.handle, e, None, 0, ctypes.byref(p), ctypes.byref(q)),
               "ctm_get_env")
        D = self.cfg.D
        shape = (p.value, q.value) if e < 8 else (p.value, D, D, q.value)
        out = np.empty(shape, dtype=np.float64)
        _check(lib.ctm_get_env(self.handle, e, out.ctypes.data, out.size, None, None),
               "ctm_get_env")
        return out

    def set_env(self, e: int, t: np.ndarray):
        t = np.ascontiguousarray(t, dtype=np.float64)
        _check(load().ctm_set_env(self.handle, e, t.ctypes.data, t.shape[0], t.shape[-1]),
               "ctm_set_env")

    def get_env_dict(self) -> dict:
        """All 16 environment tensors as {name: array} (names of ENV_NAMES)."""
        return {n: self.get_env(env_index(n)) for n in ENV_NAMES}

    def set_env_dict(self, env: dict):
        """Replace environment tensors from {name: array} (warm start)."""
        for n, t in env.items():
            self.set_env(env_index(n), t)

    @property
    def moves_done(self) -> int:
        return load().ctm_moves_done(self.handle)

    def set_precision(self, precision: int):
        _check(load().ctm_set_precision(self.handle, precision), "ctm_set_precision")
        self.cfg.precision = precision

    def set_graphs(self, enable: bool):
        _check(load().ctm_set_graphs(self.handle, int(enable)), "ctm_set_graphs")

    def profile(self, enable: bool):
        _check(load().ctm_profile(self.handle, int(enable)), "ctm_profile")

    def profile_read(self):
        """{class name: (launches, ms, flops, bytes)} for the recorded span."""
        lib = load()
        out = {}
        for i, name in enumerate(KERNEL_CLASSES):
            n = ctypes.c_longlong()
            ms, fl, by = ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
            _check(lib.ctm_profile_read(self.handle, i, ctypes.byref(n), ctypes.byref(ms),
                                        ctypes.byref(fl), ctypes.byref(by)), "ctm_profile_read")
            out[name] = (n.value, ms.value, fl.value, by.value)
        return out

    def close(self):
        if getattr(self, "_h", None) is not None:
            load().ctm_destroy(self._h)
            self._h = None
            self.workspace = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


KERNEL_CLASSES = ["gemm_f64", "gemm_f32", "gemm_bf16", "permute", "svd_round", "svd_other",
                  "reduce", "copy", "chol"]

ENV_NAMES = [f"{k}{i}{z}" for k in "CT" for i in range(1, 5) for z in "ab"]


def env_index(name: str) -> int:
    """'C1a' -> 0, ..., 'T4b' -> 15 (index = 8*kind + 2*(i-1) + z)."""
    kind = 0 if name[0] == "C" else 1
    return 8 * kind + 2 * (int(name[1]) - 1) + (0 if name[2] == "a" else 1)
