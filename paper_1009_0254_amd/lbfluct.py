"""Thin ctypes binding of liblbfluct.so (include/lbfluct.h).

Argument marshalling only: every step of the lattice Boltzmann path runs in the HIP
library.  PyTorch provides device memory (the workspace and output tensors) and the
stream.  There is no fallback: if the library is missing or the GPU is absent, the
calls raise.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np
import torch  # noqa: F401  (loads the HIP runtime the library links against)

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liblbfluct.so")

LB_OK, LB_EINVAL, LB_ENOTPSD, LB_EUNSTABLE, LB_ENOMEM, LB_EDEVICE, LB_ESTATE = 0, -1, -2, -3, -4, -5, -6
LB_FP64, LB_FP32, LB_FP32_SHIFTED = 0, 1, 2
PRECISIONS = {"fp64": LB_FP64, "fp32": LB_FP32, "fp32s": LB_FP32_SHIFTED}
INIT_KINDS = {"uniform": 0, "slab": 1, "random": 2, "wave": 3}
NOISE_KINDS = {"k0": 0, "correlated": 1, "diagonal": 2}
LB_FEATURE_STRUCTURE_FACTOR = 1
LB_SK_RESET, LB_SK_SAMPLE, LB_SK_READ, LB_SK_SNAPSHOT = 0, 1, 2, 3
LB_FLAG_CLAMPED_PIVOT, LB_FLAG_NONPOSITIVE_RHO, LB_FLAG_NAN, LB_FLAG_LOW_MACH = 1, 2, 4, 8


class LbParams(ctypes.Structure):
    _fields_ = [
        ("nx", ctypes.c_int32), ("ny", ctypes.c_int32),
        ("rho0", ctypes.c_double),
        ("rhoc", ctypes.c_double), ("A", ctypes.c_double), ("B", ctypes.c_double),
        ("kappa", ctypes.c_double), ("c0sq", ctypes.c_double),
        ("tau_bulk", ctypes.c_double), ("tau_shear", ctypes.c_double),
        ("tau_q", ctypes.c_double), ("tau_eps", ctypes.c_double),
        ("kT", ctypes.c_double),
        ("seed", ctypes.c_uint64),
        ("replica", ctypes.c_uint32),
        ("init_kind", ctypes.c_int32),
        ("noise_kind", ctypes.c_int32),
        ("reserved", ctypes.c_int32),
        ("init_arg", ctypes.c_double * 6),
    ]


class LbError(RuntimeError):
    def __init__(self, fn: str, status: int):
        super().__init__(f"{fn} failed: {status} ({lb_strerror(status)})")
        self.status = status


_lib = None


def lib() -> ctypes.CDLL:
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with python -m paper_1009_0254_amd.build")
        L = ctypes.CDLL(LIB_PATH)
        P = ctypes.POINTER(LbParams)
        vp, dp = ctypes.c_void_p, ctypes.POINTER(ctypes.c_double)
        L.lb_workspace_size.argtypes = [P, ctypes.c_int32, ctypes.c_int32, ctypes.c_uint32,
                                        ctypes.POINTER(ctypes.c_size_t)]
        L.lb_init.argtypes = [P, ctypes.c_int32, ctypes.c_int32, ctypes.c_uint32, vp, ctypes.c_size_t, vp,
                              ctypes.POINTER(vp)]
        L.lb_step.argtypes = [vp, ctypes.c_int64]
        L.lb_moments.argtypes = [vp, ctypes.c_int32, vp, dp]
        L.lb_moments_static.argtypes = [vp, ctypes.c_int32, vp, dp]
        L.lb_structure_factor.argtypes = [vp, ctypes.c_int32, ctypes.c_int32, vp, ctypes.POINTER(ctypes.c_int64)]
        L.lb_set_sampling.argtypes = [vp, ctypes.c_int64, ctypes.c_int64]
        L.lb_status_flags.argtypes = [vp, ctypes.POINTER(ctypes.c_uint32), ctypes.POINTER(ctypes.c_int64)]
        L.lb_noise_normals.argtypes = [ctypes.c_uint64, ctypes.c_uint32, ctypes.c_uint64, ctypes.c_int64,
                                       ctypes.c_int32, vp, vp]
        L.lb_philox.argtypes = [ctypes.c_uint32] * 5 + [ctypes.c_int64, vp, vp]
        L.lb_tuning.argtypes = [vp] + [ctypes.POINTER(ctypes.c_int32)] * 4
        L.lb_free.argtypes = [vp]
        L.lb_free.restype = None
        L.lb_strerror.argtypes = [ctypes.c_int32]
        L.lb_strerror.restype = ctypes.c_char_p
        for fn in ("lb_workspace_size", "lb_init", "lb_step", "lb_moments", "lb_moments_static", "lb_structure_factor",
                   "lb_set_sampling", "lb_status_flags", "lb_noise_normals", "lb_philox", "lb_tuning"):
            getattr(L, fn).restype = ctypes.c_int32
        _lib = L
    return _lib


def lb_strerror(status: int) -> str:
    return lib().lb_strerror(int(status)).decode()


def _check(fn: str, status: int):
    if status != LB_OK:
        raise LbError(fn, status)


def make_params(cfg: dict) -> LbParams:
    p = LbParams()
    p.nx, p.ny = int(cfg["nx"]), int(cfg["ny"])
    p.rho0 = float(cfg.get("rho0", 1.0))
    p.rhoc = float(cfg.get("rhoc", 1.0))
    p.A, p.B, p.kappa = float(cfg["A"]), float(cfg["B"]), float(cfg["kappa"])
    p.c0sq = float(cfg.get("c0sq", 1.0 / 3.0))
    p.tau_bulk, p.tau_shear = float(cfg["tau_bulk"]), float(cfg["tau_shear"])
    p.tau_q, p.tau_eps = float(cfg.get("tau_q", 1.0)), float(cfg.get("tau_eps", 1.0))
    p.kT = float(cfg["kT"])
    p.seed = int(cfg.get("seed", 1))
    p.replica = int(cfg.get("replica", 0))
    p.init_kind = INIT_KINDS[cfg.get("init", "uniform")]
    p.noise_kind = NOISE_KINDS[cfg.get("noise", "k0")]
    args = list(cfg.get("init_arg", [])) + [0.0] * 6
    for k in range(6):
        p.init_arg[k] = float(args[k])
    return p


def _param_array(cfgs):
    arr = (LbParams * len(cfgs))()
    for k, c in enumerate(cfgs):
        arr[k] = make_params(c)
    return arr


def lb_workspace_size(cfgs, precision: int, features: int = 0) -> int:
    arr = _param_array(cfgs)
    n = ctypes.c_size_t(0)
    _check("lb_workspace_size", lib().lb_workspace_size(arr, len(cfgs), precision, features, ctypes.byref(n)))
    return n.value


def lb_noise_normals(seed: int, replica: int, t: int, n: int, precision: int, out: torch.Tensor, stream=None):
    assert out.dtype == torch.float64 and out.is_cuda and out.numel() >= 6 * n
    s = stream if stream is not None else torch.cuda.current_stream().cuda_stream
    _check("lb_noise_normals", lib().lb_noise_normals(seed, replica, t, n, precision, out.data_ptr(), s))


def lb_philox(c1: int, c2: int, c3: int, k0: int, k1: int, n: int, out: torch.Tensor, stream=None):
    assert out.dtype == torch.int32 and out.is_cuda and out.numel() >= 4 * n
    s = stream if stream is not None else torch.cuda.current_stream().cuda_stream
    _check("lb_philox", lib().lb_philox(c1, c2, c3, k0, k1, n, out.data_ptr(), s))


class Lattice:
    """One handle: a set of replicas advanced together by the fused HIP step."""

    def __init__(self, cfgs, precision="fp32s", structure_factor=False, device="cuda:0"):
        if isinstance(cfgs, dict):
            cfgs = [cfgs]
        self.cfgs = [dict(c) for c in cfgs]
        self.precision = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
        self.features = LB_FEATURE_STRUCTURE_FACTOR if structure_factor else 0
        self.device = torch.device(device)
        self._params = _param_array(self.cfgs)
        nbytes = ctypes.c_size_t(0)
        L = lib()
        _check("lb_workspace_size", L.lb_workspace_size(self._params, len(self.cfgs), self.precision,
                                                        self.features, ctypes.byref(nbytes)))
        self.workspace = torch.empty(nbytes.value + 256, dtype=torch.uint8, device=self.device)
        base = self.workspace.data_ptr()
        self._ws_ptr = (base + 255) // 256 * 256
        self.stream = torch.cuda.current_stream(self.device)
        h = ctypes.c_void_p()
        _check("lb_init", L.lb_init(self._params, len(self.cfgs), self.precision, self.features,
                                    self._ws_ptr, nbytes.value, self.stream.cuda_stream, ctypes.byref(h)))
        self._h = h

    # -- ABI calls ---------------------------------------------------------------------
    def lb_step(self, nsteps: int):
        _check("lb_step", lib().lb_step(self._h, int(nsteps)))

    def lb_moments(self, rep: int = 0, planes: bool = True):
        c = self.cfgs[rep]
        m = torch.empty((9, c["ny"], c["nx"]), dtype=torch.float64, device=self.device) if planes else None
        tot = (ctypes.c_double * 6)()
        _check("lb_moments", lib().lb_moments(self._h, rep, m.data_ptr() if planes else None, tot))
        return m, np.array(tot[:])

    def lb_moments_static(self, rep: int = 0, planes: bool = True):
        c = self.cfgs[rep]
        m = torch.empty((9, c["ny"], c["nx"]), dtype=torch.float64, device=self.device) if planes else None
        tot = (ctypes.c_double * 6)()
        _check("lb_moments_static", lib().lb_moments_static(self._h, rep, m.data_ptr() if planes else None, tot))
        return m, np.array(tot[:])

    def lb_structure_factor(self, op: int, rep: int = -1):
        if op == LB_SK_SNAPSHOT:
            nb = ctypes.c_int64(0)
            _check("lb_structure_factor", lib().lb_structure_factor(self._h, op, rep, None, ctypes.byref(nb)))
            out = torch.empty((2, nb.value), dtype=torch.float64, device=self.device)
            _check("lb_structure_factor", lib().lb_structure_factor(self._h, op, rep, out.data_ptr(), ctypes.byref(nb)))
            return out
        if op == LB_SK_READ:
            c = self.cfgs[rep]
            out = torch.empty((9, c["ny"], c["nx"] // 2 + 1), dtype=torch.float64, device=self.device)
            ns = ctypes.c_int64(0)
            _check("lb_structure_factor", lib().lb_structure_factor(self._h, op, rep, out.data_ptr(), ctypes.byref(ns)))
            return out, ns.value
        _check("lb_structure_factor", lib().lb_structure_factor(self._h, op, rep, None, None))
        return None

    def lb_set_sampling(self, every: int, first_step: int = 0):
        _check("lb_set_sampling", lib().lb_set_sampling(self._h, int(every), int(first_step)))

    def lb_status_flags(self):
        f = ctypes.c_uint32(0)
        t = ctypes.c_int64(0)
        _check("lb_status_flags", lib().lb_status_flags(self._h, ctypes.byref(f), ctypes.byref(t)))
        return f.value, t.value

    def lb_tuning(self):
        """(strip width, rows per tile, workgroups, steps per launch)"""
        v = [ctypes.c_int32(0) for _ in range(4)]
        _check("lb_tuning", lib().lb_tuning(self._h, *[ctypes.byref(x) for x in v]))
        return tuple(x.value for x in v)

    # -- conveniences ------------------------------------------------------------------
    step = lb_step

    def moments(self, rep: int = 0) -> np.ndarray:
        m, _ = self.lb_moments(rep, True)
        return m.cpu().numpy()

    def totals(self, rep: int = 0) -> np.ndarray:
        return self.lb_moments(rep, False)[1]

    def close(self):
        if getattr(self, "_h", None):
            lib().lb_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
