"""ctypes binding of libhps.so (the C-ABI declared in include/hps.h).

Argument marshalling only: every step of the operator, the preconditioner and
the solvers runs in the library's HIP kernels.  torch provides device memory
(complex128 tensors) and the current stream.  The binding refuses to run
without the compiled library; there is no fallback.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libhps.so")

HPS_OK = 0
HPS_NOT_CONVERGED = 1
HPS_ERR_ARG, HPS_ERR_UNSUPPORTED, HPS_ERR_OOM = -1, -2, -3
HPS_ERR_DEVICE, HPS_ERR_BREAKDOWN, HPS_ERR_NUMERIC = -4, -5, -6
ERRORS = {-1: "ARG", -2: "UNSUPPORTED", -3: "OOM", -4: "DEVICE", -5: "BREAKDOWN", -6: "NUMERIC"}
PREC = {"fp64": 1, "fp32": 2, "bf16": 4, "separable": 8}
SOLVER = {"gmres": 0, "fgmres": 1, "batched": 2, "iti": 3, "block_gmres": 4, "ir": 5}
ORTH = {"dcgs": 0, "cgs2": 1}
MEDIUM_ZERO, MEDIUM_NODAL, MEDIUM_BUMPS = 0, 1, 2


class HPSError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"hps error {code} ({ERRORS.get(code, '?')}): {msg}")
        self.code = code


class _Z(ctypes.Structure):
    _fields_ = [("re", ctypes.c_double), ("im", ctypes.c_double)]


class _Domain(ctypes.Structure):
    _fields_ = [("lo", ctypes.c_double * 3), ("hi", ctypes.c_double * 3)]


class _Medium(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int), ("n_bumps", ctypes.c_int),
                ("centres", ctypes.POINTER(ctypes.c_double)), ("amps", ctypes.POINTER(_Z)),
                ("width", ctypes.c_double), ("nodal", ctypes.c_void_p)]


class _Opts(ctypes.Structure):
    _fields_ = [("block_precs", ctypes.c_int), ("stream", ctypes.c_void_p), ("verbose", ctypes.c_int),
                ("lambda_bucket", ctypes.c_double)]


class _SolveOpts(ctypes.Structure):
    _fields_ = [("solver", ctypes.c_int), ("max_iters", ctypes.c_int), ("use_x0", ctypes.c_int),
                ("precond_prec", ctypes.c_int), ("check_every", ctypes.c_int), ("orth", ctypes.c_int),
                ("rhs_rel_res", ctypes.POINTER(ctypes.c_double)), ("inner_tol", ctypes.c_double)]


class Stats(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int), ("restarts", ctypes.c_int), ("converged", ctypes.c_int),
                ("lambda_shifted", ctypes.c_int), ("rel_res", ctypes.c_double),
                ("true_rel_res", ctypes.c_double), ("t_setup", ctypes.c_double),
                ("t_solve", ctypes.c_double),
                ("bytes_apply", ctypes.c_double), ("bytes_precond", ctypes.c_double)]

    def as_dict(self) -> dict:
        return {k: getattr(self, k) for k, _ in self._fields_}


# exported symbols and their signatures
SIGNATURES = {
    "hps_setup": (ctypes.c_int, [ctypes.POINTER(_Domain), ctypes.c_double, ctypes.c_double,
                                 ctypes.POINTER(_Medium), ctypes.c_int, ctypes.c_int,
                                 ctypes.POINTER(ctypes.c_int), ctypes.POINTER(_Opts),
                                 ctypes.POINTER(ctypes.c_void_p)]),
    "hps_setup_group": (ctypes.c_int, [ctypes.POINTER(_Domain), ctypes.c_int, ctypes.POINTER(ctypes.c_double),
                                       ctypes.POINTER(ctypes.c_double), ctypes.c_void_p, ctypes.c_int,
                                       ctypes.c_int, ctypes.POINTER(ctypes.c_int), ctypes.POINTER(_Opts),
                                       ctypes.POINTER(ctypes.c_void_p)]),
    "hps_num_operators": (ctypes.c_int, [ctypes.c_void_p]),
    "hps_num_unknowns": (ctypes.c_int64, [ctypes.c_void_p]),
    "hps_num_blocks": (ctypes.c_int64, [ctypes.c_void_p]),
    "hps_nodes": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_double)]),
    "hps_lambdas": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(_Z)]),
    "hps_set_stream": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p]),
    "hps_apply": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int]),
    "hps_apply_noalloc": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int]),
    "hps_op_left_f32": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int]),
    "hps_precond_f32": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int]),
    "hps_precond": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int]),
    "hps_op_left": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int]),
    "hps_autotune": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                    ctypes.POINTER(ctypes.c_int)]),
    "hps_autotune_set": (ctypes.c_int, [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int]),
    "hps_autotune_get": (ctypes.c_int, [ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                        ctypes.POINTER(ctypes.c_int)]),
    "hps_autotune_save": (ctypes.c_int, [ctypes.c_char_p]),
    "hps_autotune_load": (ctypes.c_int, [ctypes.c_char_p]),
    "hps_iti_build": (ctypes.c_int, [ctypes.c_void_p]),
    "hps_iti_apply": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int]),
    "hps_iti_rhs": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                   ctypes.c_int]),
    "hps_iti_recover": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                       ctypes.c_void_p, ctypes.c_int]),
    "hps_iti_bytes": (ctypes.c_int64, [ctypes.c_int, ctypes.POINTER(ctypes.c_int)]),
    "hps_precond_prec": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                        ctypes.c_int, ctypes.c_int]),
    "hps_assemble_rhs": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                        ctypes.c_void_p, ctypes.c_int]),
    "hps_gmres": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_double,
                                 ctypes.c_int, ctypes.c_void_p, ctypes.c_int,
                                 ctypes.POINTER(_SolveOpts), ctypes.POINTER(Stats)]),
    "hps_device_bytes": (ctypes.c_int64, [ctypes.c_void_p]),
    "hps_set_timing": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int]),
    "hps_separable_table": (ctypes.c_int, [ctypes.c_int, ctypes.c_double, ctypes.c_double,
                                           ctypes.POINTER(ctypes.c_double)]),
    "hps_arnoldi_times": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_double), ctypes.c_int]),
    "hps_kernel_times": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_double), ctypes.c_int]),
    "hps_setup_bytes": (ctypes.c_int64, [ctypes.c_int, ctypes.POINTER(ctypes.c_int), ctypes.c_int,
                                         ctypes.c_int, ctypes.POINTER(ctypes.c_int64)]),
    "hps_solve_bytes": (ctypes.c_int64, [ctypes.c_void_p, ctypes.c_int, ctypes.c_int,
                                         ctypes.POINTER(_SolveOpts)]),
    "hps_trim": (ctypes.c_int, [ctypes.c_void_p]),
    "hps_last_error": (ctypes.c_char_p, []),
    "hps_free": (None, [ctypes.c_void_p]),
}

_lib = None


def lib() -> ctypes.CDLL:
    """Load libhps.so; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                               "`python -m paper_2112_02211_amd.build` (no fallback exists)")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def _check(rc: int, allow_nc: bool = False) -> int:
    if rc == HPS_OK or (allow_nc and rc == HPS_NOT_CONVERGED):
        return rc
    raise HPSError(rc, lib().hps_last_error().decode())


def _torch():
    import torch
    return torch


def _stream_ptr():
    torch = _torch()
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _dev_opt(t, name: str):
    """_dev, or NULL for None (optional arguments such as zero boundary data)."""
    return None if t is None else _dev(t, name)


def _dev32(t, name: str):
    torch = _torch()
    if not isinstance(t, torch.Tensor) or t.device.type != "cuda" or t.dtype != torch.complex64:
        raise TypeError(f"{name} must be a complex64 CUDA tensor")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    return ctypes.c_void_p(t.data_ptr())


def _dev(t, name: str):
    torch = _torch()
    if not isinstance(t, torch.Tensor) or t.device.type != "cuda" or t.dtype != torch.complex128:
        raise TypeError(f"{name} must be a complex128 CUDA tensor")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    return ctypes.c_void_p(t.data_ptr())


class Context:
    """One discretized problem resident on the GPU (tables, medium, blocks)."""

    def __init__(self, n_elem: Sequence[int], p: int, kappa: float, eta: Optional[float] = None,
                 lo=(0.0, 0.0, 0.0), hi=None, bump_centres=None, bump_amps=None,
                 bump_width: float = 0.08, nodal_b=None, block_precs=("fp64",),
                 q: Optional[int] = None, verbose: bool = False, lambda_bucket: float = 0.0):
        """lambda_bucket = delta > 0 rounds each leaf's homogenized lambda to a
        grid of spacing delta kappa^2 and builds one block per distinct rounded
        value (leaves that share it share the block); 0 builds one per leaf."""
        L = lib()
        self.n_elem = tuple(int(e) for e in n_elem)
        self.p = int(p)
        self.kappa = float(kappa)
        self.eta = float(kappa if eta is None else eta)
        if hi is None:
            m = float(max(self.n_elem))
            hi = tuple(float(e) / m for e in self.n_elem)
        dom = _Domain((ctypes.c_double * 3)(*lo), (ctypes.c_double * 3)(*hi))
        self._keep = []
        med = _Medium()
        _fill_medium(med, self._keep, bump_centres, bump_amps, bump_width, nodal_b)
        bits = 0
        for name in block_precs:
            bits |= PREC[name]
        self.block_precs = tuple(block_precs)
        self.lambda_bucket = float(lambda_bucket)
        opts = _Opts(bits, _stream_ptr(), 1 if verbose else 0, self.lambda_bucket)
        ne = (ctypes.c_int * 3)(*self.n_elem)
        handle = ctypes.c_void_p()
        qq = self.p - 2 if q is None else int(q)
        _check(L.hps_setup(ctypes.byref(dom), self.kappa, self.eta, ctypes.byref(med), self.p, qq,
                           ne, ctypes.byref(opts), ctypes.byref(handle)))
        self._attach(handle)

    def _attach(self, handle):
        L = lib()
        self._h = handle
        self.N = int(L.hps_num_unknowns(handle))
        n1 = self.p - 2
        self.ni, self.nb = n1 ** 3, 6 * n1 * n1
        self.n = self.ni + self.nb
        self.nl = int(np.prod(self.n_elem))
        self.n_blocks = int(L.hps_num_blocks(handle))
        self.n_ops = int(L.hps_num_operators(handle))

    @classmethod
    def group(cls, probs, block_precs=("fp64",), verbose: bool = False) -> "Context":
        """One context for several problems on the same mesh (n_elem, p, box)
        with their own kappa, eta and medium: every launch covers all of them,
        and vectors hold one right-hand side per problem ([op][N])."""
        L = lib()
        p0 = probs[0]
        for pr in probs[1:]:
            if (tuple(pr.n_elem), pr.p, tuple(pr.lo), tuple(pr.hi)) != (tuple(p0.n_elem), p0.p, tuple(p0.lo),
                                                                       tuple(p0.hi)):
                raise ValueError("a group needs the same mesh (n_elem, p, box) for every problem")
        self = cls.__new__(cls)
        self.n_elem = tuple(int(e) for e in p0.n_elem)
        self.p = int(p0.p)
        self.kappa = float(p0.kappa)
        self.eta = float(p0.eta)
        self.lambda_bucket = 0.0
        self._keep = []
        k = len(probs)
        meds = (_Medium * k)()
        for i, pr in enumerate(probs):
            if pr.plane_dir is not None or len(pr.bump_centres) == 0:
                _fill_medium(meds[i], self._keep, None, None, 0.08, None)
            else:
                _fill_medium(meds[i], self._keep, pr.bump_centres, pr.bump_amps, pr.bump_width, None)
        bits = 0
        for name in block_precs:
            bits |= PREC[name]
        self.block_precs = tuple(block_precs)
        kap = (ctypes.c_double * k)(*[float(pr.kappa) for pr in probs])
        eta = (ctypes.c_double * k)(*[float(pr.eta) for pr in probs])
        dom = _Domain((ctypes.c_double * 3)(*p0.lo), (ctypes.c_double * 3)(*p0.hi))
        opts = _Opts(bits, _stream_ptr(), 1 if verbose else 0, 0.0)
        ne = (ctypes.c_int * 3)(*self.n_elem)
        handle = ctypes.c_void_p()
        _check(L.hps_setup_group(ctypes.byref(dom), k, kap, eta, ctypes.cast(meds, ctypes.c_void_p), self.p,
                                 self.p - 2, ne, ctypes.byref(opts), ctypes.byref(handle)))
        self._keep.append(meds)
        self._attach(handle)
        return self

    @classmethod
    def from_problem(cls, prob, block_precs=("fp64",), verbose=False,
                     lambda_bucket: Optional[float] = None) -> "Context":
        """Context for a problems.Problem (bump medium, or b = 0 for plane waves);
        lambda_bucket defaults to the problem's own."""
        if lambda_bucket is None:
            lambda_bucket = getattr(prob, "lambda_bucket", 0.0)
        if prob.plane_dir is not None or len(prob.bump_centres) == 0:
            return cls(prob.n_elem, prob.p, prob.kappa, prob.eta, prob.lo, prob.hi,
                       block_precs=block_precs, verbose=verbose, lambda_bucket=lambda_bucket)
        return cls(prob.n_elem, prob.p, prob.kappa, prob.eta, prob.lo, prob.hi,
                   bump_centres=prob.bump_centres, bump_amps=prob.bump_amps,
                   bump_width=prob.bump_width, block_precs=block_precs, verbose=verbose,
                   lambda_bucket=lambda_bucket)

    # ------------------------------------------------------------------ info
    def _sync_stream(self):
        _check(lib().hps_set_stream(self._h, _stream_ptr()))

    def nodes(self) -> np.ndarray:
        out = np.zeros((self.N, 3), dtype=np.float64)
        _check(lib().hps_nodes(self._h, out.ctypes.data_as(ctypes.POINTER(ctypes.c_double))))
        return out

    def lambdas(self) -> np.ndarray:
        self._sync_stream()
        out = np.zeros(self.nl * getattr(self, "n_ops", 1), dtype=np.complex128)
        _check(lib().hps_lambdas(self._h, out.ctypes.data_as(ctypes.POINTER(_Z))))
        return out

    def set_timing(self, enable=True, every: int = 1):
        """Event timing of every `every`-th apply / J^-1 / GEMM launch (off if not enable)."""
        self._sync_stream()
        _check(lib().hps_set_timing(self._h, int(every) if enable else 0))

    def kernel_times(self, reset: bool = False) -> dict:
        """Event-timed operator / preconditioner launches since the last reset."""
        out = (ctypes.c_double * 8)()
        _check(lib().hps_kernel_times(self._h, out, 1 if reset else 0))
        return {"apply_ms": out[0], "apply_launches": int(out[1]),
                "precond_ms": out[2], "precond_launches": int(out[3]),
                "gemm_ms": out[4], "gemm_launches": int(out[5]),
                "iti_ms": out[6], "iti_launches": int(out[7])}

    def arnoldi_times(self, reset: bool = False) -> dict:
        """Event-timed Arnoldi update passes since the last reset, with their
        algorithmic HBM bytes."""
        out = (ctypes.c_double * 3)()
        _check(lib().hps_arnoldi_times(self._h, out, 1 if reset else 0))
        return {"update_ms": out[0], "update_launches": int(out[1]), "update_bytes": out[2]}

    def solve_bytes(self, restart: int, nrhs: int = 1, solver: str = "gmres",
                    precond_prec: str = "fp64") -> int:
        """Device bytes a gmres call with these settings needs (library's own plan)."""
        so = _SolveOpts(SOLVER[solver], 0, 0, PREC[precond_prec], 1, 0)
        v = int(lib().hps_solve_bytes(self._h, int(restart), int(nrhs), ctypes.byref(so)))
        if v < 0:
            raise HPSError(v, lib().hps_last_error().decode())
        return v

    def trim(self):
        """Free the solver/operator workspaces (blocks stay resident)."""
        self._sync_stream()
        _check(lib().hps_trim(self._h))

    def device_bytes(self) -> int:
        return int(lib().hps_device_bytes(self._h))

    # ------------------------------------------------------------- operators
    def _nrhs(self, x) -> int:
        if x.numel() % self.N:
            raise ValueError("vector length is not a multiple of N")
        return x.numel() // self.N

    def apply(self, x, y=None):
        """y = A x for nrhs = x.numel() / N vectors stored one after the other."""
        torch = _torch()
        y = torch.empty_like(x) if y is None else y
        self._sync_stream()
        _check(lib().hps_apply(self._h, _dev(x, "x"), _dev(y, "y"), self._nrhs(x)))
        return y

    def op_left_f32(self, x, y=None):
        """y = J^{-1} A x on complex64 vectors (the inner operator of iterative refinement)."""
        torch = _torch()
        y = torch.empty_like(x) if y is None else y
        self._sync_stream()
        _check(lib().hps_op_left_f32(self._h, _dev32(x, "x"), _dev32(y, "y"), self._nrhs(x)))
        return y

    def precond_f32(self, x, y=None):
        """y = J^{-1} x on complex64 vectors (separable form)."""
        torch = _torch()
        y = torch.empty_like(x) if y is None else y
        self._sync_stream()
        _check(lib().hps_precond_f32(self._h, _dev32(x, "x"), _dev32(y, "y"), self._nrhs(x)))
        return y

    def apply_noalloc(self, x, y):
        """y = A x with the face buffer in the library's static device array:
        the call allocates no device memory (y must be given)."""
        self._sync_stream()
        _check(lib().hps_apply_noalloc(self._h, _dev(x, "x"), _dev(y, "y"), self._nrhs(x)))
        return y

    def precond(self, x, y=None, prec: str = "fp64"):
        """y = J^{-1} x with the blocks stored in ``prec``."""
        torch = _torch()
        y = torch.empty_like(x) if y is None else y
        self._sync_stream()
        _check(lib().hps_precond_prec(self._h, _dev(x, "x"), _dev(y, "y"), self._nrhs(x), PREC[prec]))
        return y

    def op_left(self, x, y=None):
        """y = J^{-1} A x (FP64 blocks): the left-preconditioned operator."""
        torch = _torch()
        y = torch.empty_like(x) if y is None else y
        self._sync_stream()
        _check(lib().hps_op_left(self._h, _dev(x, "x"), _dev(y, "y"), self._nrhs(x)))
        return y

    # ------------------------------------------------- face-reduced system
    def iti_build(self):
        """Form the exact ItI map R and A_ii^{-1} of every leaf (face-reduced system)."""
        self._sync_stream()
        _check(lib().hps_iti_build(self._h))

    def _nrhs_face(self, f) -> int:
        nf = self.nl * self.nb
        if f.numel() % nf:
            raise ValueError(f"face vector length {f.numel()} is not a multiple of N_l n_b = {nf}")
        return f.numel() // nf

    def iti_apply(self, f, y=None):
        """y = f + Pi (R f): the face-reduced operator."""
        torch = _torch()
        y = torch.empty_like(f) if y is None else y
        self._sync_stream()
        _check(lib().hps_iti_apply(self._h, _dev(f, "f"), _dev(y, "y"), self._nrhs_face(f)))
        return y

    def iti_rhs(self, s, t):
        """t - Pi h: the right-hand side of the face-reduced system."""
        torch = _torch()
        nrhs = self._nrhs(s)
        out = torch.empty(nrhs * self.nl * self.nb, dtype=s.dtype, device=s.device)
        self._sync_stream()
        _check(lib().hps_iti_rhs(self._h, _dev(s, "s"), _dev_opt(t, "t"), _dev(out, "rhs_f"), nrhs))
        return out

    def iti_recover(self, s, t, f):
        """u from the incoming impedance f (leaf solves with source s)."""
        torch = _torch()
        u = torch.empty_like(s)
        self._sync_stream()
        _check(lib().hps_iti_recover(self._h, _dev(s, "s"), _dev_opt(t, "t"), _dev(f, "f"), _dev(u, "u"),
                                     self._nrhs(s)))
        return u

    def autotune(self, nrhs: int, prec: str = "fp32", reps: int = 3) -> int:
        """Time the block-GEMM tile shapes on this operator for nrhs right-hand
        sides and record the fastest (process-wide); returns its index."""
        self._sync_stream()
        out = ctypes.c_int(-1)
        _check(lib().hps_autotune(self._h, int(nrhs), PREC[prec], int(reps), ctypes.byref(out)))
        return out.value

    def assemble_rhs(self, s, t, b=None):
        torch = _torch()
        b = torch.empty_like(s) if b is None else b
        self._sync_stream()
        _check(lib().hps_assemble_rhs(self._h, _dev(s, "s"), _dev_opt(t, "t"), _dev(b, "b"),
                                      self._nrhs(s)))
        return b

    def gmres(self, s, t, tol: float = 1e-10, restart: int = 30, u=None, solver: str = "gmres",
              precond_prec: str = "fp64", max_iters: int = 0, check_every: int = 1,
              use_x0: bool = False, raise_on_nc: bool = False, orth: str = "dcgs",
              inner_tol: float = 0.0):
        """Solve A u = b(s, t); returns (u, stats dict, converged flag).
        t may be None: zero boundary data.

        orth: "dcgs" (delayed reorthogonalization, two passes per step; restart
        <= 64) or "cgs2" (classical Gram-Schmidt twice, three passes).
        solver "ir": iterative refinement with FP32 inner solves stopped at
        inner_tol (0: the library's default)."""
        torch = _torch()
        u = torch.zeros_like(s) if u is None else u
        nrhs = self._nrhs(s)
        res = (ctypes.c_double * nrhs)()
        so = _SolveOpts(SOLVER[solver], int(max_iters), 1 if use_x0 else 0,
                        0 if solver == "ir" else PREC[precond_prec], int(check_every), ORTH[orth],
                        ctypes.cast(res, ctypes.POINTER(ctypes.c_double)), float(inner_tol))
        st = Stats()
        self._sync_stream()
        rc = lib().hps_gmres(self._h, _dev(s, "s"), _dev_opt(t, "t"), float(tol), int(restart),
                             _dev(u, "u"), nrhs, ctypes.byref(so), ctypes.byref(st))
        _check(rc, allow_nc=not raise_on_nc)
        d = st.as_dict()
        d["rhs_rel_res"] = list(res)          # final relative residual of each right-hand side
        return u, d, rc == HPS_OK

    def free(self):
        if getattr(self, "_h", None):
            lib().hps_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


def _fill_medium(med, keep, bump_centres, bump_amps, bump_width, nodal_b):
    """Fill an hps_medium: nodal b (device tensor), Gaussian bumps, or zero."""
    if nodal_b is not None:
        med.kind = MEDIUM_NODAL
        med.nodal = _dev(nodal_b, "nodal_b")
        keep.append(nodal_b)
    elif bump_centres is not None and len(bump_centres) > 0:
        c = np.ascontiguousarray(np.asarray(bump_centres, dtype=np.float64).reshape(-1, 3))
        a = np.asarray(bump_amps, dtype=np.complex128)
        za = (_Z * len(a))(*[_Z(float(v.real), float(v.imag)) for v in a])
        med.kind = MEDIUM_BUMPS
        med.n_bumps = len(a)
        med.centres = c.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
        med.amps = za
        med.width = float(bump_width)
        keep += [c, za]
    else:
        med.kind = MEDIUM_ZERO


def iti_bytes(n_elem, p) -> int:
    """Device bytes hps_iti_build keeps for this mesh (no GPU needed)."""
    ne = (ctypes.c_int * 3)(*[int(e) for e in n_elem])
    v = int(lib().hps_iti_bytes(int(p), ne))
    if v < 0:
        raise HPSError(v, lib().hps_last_error().decode())
    return v


def separable_table(p: int, h: float, eta: float):
    """(Wc, Vc, Ec, Fi) of the separable J^-1 for a leaf of side h (host only)."""
    n1 = int(p) - 2
    out = np.zeros(2 * (2 * n1 * n1 + n1 + 4))
    _check(lib().hps_separable_table(int(p), float(h), float(eta),
                                     out.ctypes.data_as(ctypes.POINTER(ctypes.c_double))))
    z = out[0::2] + 1j * out[1::2]
    L = n1 * n1
    return (z[:L].reshape(n1, n1), z[L:2 * L].reshape(n1, n1), z[2 * L:2 * L + n1],
            z[2 * L + n1:].reshape(2, 2))


def setup_bytes(n_elem, p, block_precs=("fp64",), complex_medium=False):
    """(resident, transient) device bytes of hps_setup for this mesh (no GPU needed)."""
    bits = 0
    for name in block_precs:
        bits |= PREC[name]
    tr = ctypes.c_int64()
    ne = (ctypes.c_int * 3)(*[int(e) for e in n_elem])
    v = int(lib().hps_setup_bytes(int(p), ne, bits, 1 if complex_medium else 0, ctypes.byref(tr)))
    if v < 0:
        raise HPSError(v, lib().hps_last_error().decode())
    return v, int(tr.value)


def setup_error(n_elem, p, q, kappa=10.0, lo=(0, 0, 0), hi=(1, 1, 1)):
    """Run hps_setup on arguments expected to be rejected; returns (code, message).

    The argument checks happen before any device call, so this runs without a GPU.
    """
    L = lib()
    dom = _Domain((ctypes.c_double * 3)(*lo), (ctypes.c_double * 3)(*hi))
    ne = (ctypes.c_int * 3)(*n_elem)
    h = ctypes.c_void_p()
    rc = L.hps_setup(ctypes.byref(dom), float(kappa), float(kappa), None, int(p), int(q), ne, None,
                     ctypes.byref(h))
    if rc == HPS_OK:
        L.hps_free(h)
    return rc, L.hps_last_error().decode()


GEMM_SHAPES = [(8, 64), (8, 32), (8, 16), (4, 64), (4, 32), (4, 16)]   # (wavefronts, panel)


def autotune_set(p: int, prec: str, nrhs: int, shape: int):
    """Record (or with shape = -1 remove) the block-GEMM tile shape for (p, prec, nrhs)."""
    _check(lib().hps_autotune_set(int(p), PREC[prec], int(nrhs), int(shape)))


def autotune_get(p: int, prec: str, nrhs: int) -> int:
    out = ctypes.c_int(-1)
    _check(lib().hps_autotune_get(int(p), PREC[prec], int(nrhs), ctypes.byref(out)))
    return out.value


def autotune_save(path: str):
    _check(lib().hps_autotune_save(os.fsencode(path)))


def autotune_load(path: str):
    _check(lib().hps_autotune_load(os.fsencode(path)))
