"""MI355X (gfx950) library for the shift-invariant parameter-to-observable
map of arXiv 2504.16344: Python binding over the C ABI in include/p2o.h.

This module only marshals arguments (device pointers from torch tensors and
the current HIP stream) into libp2o.so; every step of the computation runs in
the library's HIP kernels.  Importing works without a GPU; using a Plan
requires the built library and a GPU, and raises if either is missing.
"""
from __future__ import annotations

import ctypes
import os

import torch

__all__ = [
    "Plan", "Batch", "Graph", "P2OError", "P2OApply", "P2OAdjoint", "load_library", "LIB_PATH",
    "FP64", "MIXED", "FAST", "MIXED_FP16", "MIXED_BF16", "FAST_BF16", "OP_F", "OP_FADJ",
    "smooth_length", "EXPORTED_SYMBOLS", "qoi_predict",
]

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libp2o.so")

# p2o_prec: P2O_MIXED is the bfloat16 hi+lo tier, P2O_FAST the bfloat16 hi-only one
FP64, MIXED, FAST, MIXED_FP16 = 0, 1, 2, 3
MIXED_BF16, FAST_BF16 = MIXED, FAST
PREC_BY_NAME = {"fp64": FP64, "mixed": MIXED, "fast": FAST, "mixed_bf16": MIXED_BF16,
                "fast_bf16": FAST_BF16, "mixed_fp16": MIXED_FP16}
OP_F, OP_FADJ = 0, 1
ASSEMBLY = {"matvec": 0, "gram": 1}  # p2o_assembly

STATUS = {0: "P2O_OK", 1: "P2O_EINVAL", 2: "P2O_ENOMEM", 3: "P2O_EHIP",
          4: "P2O_ENOTPD", 5: "P2O_ESTATE", 6: "P2O_EUNSUPPORTED"}

_c = ctypes
_vp, _i64, _int, _dbl = _c.c_void_p, _c.c_int64, _c.c_int, _c.c_double


class _PriorGrid(_c.Structure):
    """p2o_prior_grid of include/p2o.h."""
    _fields_ = [("nx", _i64), ("ny", _i64), ("radius", _int), ("length", _dbl),
                ("delta", _dbl)]


_SIGNATURES = {
    "p2o_setup": (_int, [_vp, _i64, _i64, _i64, _int, _vp, _c.POINTER(_vp)]),
    "p2o_setup_begin": (_int, [_i64, _i64, _i64, _int, _vp, _c.POINTER(_vp)]),
    "p2o_setup_columns": (_int, [_vp, _vp, _i64, _i64, _vp]),
    "p2o_setup_end": (_int, [_vp, _vp]),
    "p2o_get_info": (_int, [_vp, _c.POINTER(_i64), _c.POINTER(_i64), _c.POINTER(_i64),
                            _c.POINTER(_i64), _c.POINTER(_int)]),
    "p2o_reserve": (_int, [_vp, _i64, _vp]),
    "p2o_apply": (_int, [_vp, _int, _vp, _vp, _i64, _vp]),
    "p2o_hessian_assemble": (_int, [_vp, _dbl, _vp, _vp, _vp]),
    "p2o_posterior_solve": (_int, [_vp, _vp, _vp, _vp, _i64, _dbl, _int,
                                   _c.POINTER(_i64), _vp]),
    "p2o_qoi_precompute": (_int, [_vp, _vp, _vp, _dbl, _vp, _vp, _vp]),
    "p2o_set_prior": (_int, [_vp, _c.POINTER(_PriorGrid), _vp]),
    "p2o_set_assembly": (_int, [_vp, _int]),
    "p2o_posterior_mean": (_int, [_vp, _vp, _vp, _vp, _i64, _dbl, _vp]),
    "p2o_posterior_invert": (_int, [_vp, _vp, _vp, _vp]),
    "p2o_posterior_mean_kinv": (_int, [_vp, _vp, _vp, _vp, _i64, _dbl, _vp]),
    "p2o_posterior_mean_kinv_noalloc": (_int, [_vp, _vp, _vp, _vp, _i64, _dbl, _vp]),
    "p2o_read_bandwidth": (_int, [_vp, _i64, _vp, _vp]),
    "p2o_qoi_predict": (_int, [_vp, _i64, _i64, _vp, _vp, _i64, _vp]),
    "p2o_destroy": (None, [_vp]),
    "p2o_status_string": (_c.c_char_p, [_int]),
    "p2o_last_hip_error": (_int, [_c.POINTER(_int)]),
    "p2o_set_kernel_timing": (_int, [_vp, _int]),
    "p2o_autotune": (_int, [_vp, _int, _int, _c.POINTER(_dbl), _i64, _c.POINTER(_i64), _vp]),
    "p2o_get_config": (_int, [_vp, _int, _c.POINTER(_i64), _c.POINTER(_i64)]),
    "p2o_set_config": (_int, [_vp, _int, _i64]),
    "p2o_set_mfma_threshold": (_int, [_vp, _int, _i64]),
    "p2o_kernel_time": (_int, [_vp, _int, _c.POINTER(_dbl), _c.POINTER(_i64)]),
    "p2o_batch_create": (_int, [_c.POINTER(_vp), _i64, _c.POINTER(_vp)]),
    "p2o_batch_apply": (_int, [_vp, _int, _c.POINTER(_vp), _c.POINTER(_vp), _c.POINTER(_i64), _vp]),
    "p2o_graph_capture": (_int, [_vp, _int, _c.POINTER(_vp), _c.POINTER(_vp), _c.POINTER(_i64),
                                 _vp, _c.POINTER(_vp)]),
    "p2o_batch_capture": (_int, [_vp, _int, _c.POINTER(_vp), _c.POINTER(_vp), _c.POINTER(_i64),
                                 _vp, _c.POINTER(_vp)]),
    "p2o_graph_launch": (_int, [_vp, _vp]),
    "p2o_graph_destroy": (None, [_vp]),
    "p2o_batch_destroy": (None, [_vp]),
    "p2o_batch_autotune": (_int, [_vp, _int, _c.POINTER(_vp), _c.POINTER(_vp), _c.POINTER(_i64),
                                  _int, _c.POINTER(_dbl), _i64, _c.POINTER(_i64), _vp]),
    "p2o_batch_set_config": (_int, [_vp, _int, _i64]),
    "p2o_batch_get_config": (_int, [_vp, _int, _c.POINTER(_i64), _c.POINTER(_i64)]),
}
EXPORTED_SYMBOLS = tuple(_SIGNATURES)

_lib = None


def load_library(path: str = LIB_PATH):
    """Load libp2o.so and declare its signatures.  Raises if it is not built."""
    global _lib
    if _lib is not None and path == LIB_PATH:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(
            f"{path} is missing: the HIP library has not been built "
            "(run __graft_entry__.build()); there is no fallback path")
    lib = ctypes.CDLL(path)
    for name, (res, args) in _SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    if path == LIB_PATH:
        _lib = lib
    return lib


class P2OError(RuntimeError):
    def __init__(self, call: str, status: int):
        lib = load_library()
        hip = _c.c_int(0)
        lib.p2o_last_hip_error(_c.byref(hip))
        msg = lib.p2o_status_string(status).decode()
        extra = f" (HIP error {hip.value})" if status == 3 else ""
        super().__init__(f"{call} -> {STATUS.get(status, status)}: {msg}{extra}")
        self.status = status
        self.hip_error = hip.value if status == 3 else 0


def _check(call: str, status: int) -> None:
    if status != 0:
        raise P2OError(call, status)


def smooth_length(Nt: int) -> int:
    """Embedding length L: smallest even integer >= 2*Nt with prime factors in {2,3,5,7}."""
    L = 2 * Nt
    while True:
        n = L
        for p in (2, 3, 5, 7):
            while n % p == 0:
                n //= p
        if n == 1:
            return L
        L += 2


def _stream_handle(stream) -> int:
    if stream is None:
        stream = torch.cuda.current_stream()
    return stream.cuda_stream if hasattr(stream, "cuda_stream") else int(stream)


def _dev_f64(t: torch.Tensor, name: str) -> torch.Tensor:
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a CUDA (HIP) tensor")
    if t.dtype != torch.float64:
        raise TypeError(f"{name} must be float64, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    return t


class Plan:
    """A set-up p2o map: frequency blocks resident on the current GPU.

    ``Plan(blocks, prec)`` runs p2o_setup on a [Nt][Nd][Nm] float64 CUDA
    tensor.  ``Plan.begin(Nd, Nm, Nt, prec)`` starts a chunked setup
    (``setup_columns`` then ``setup_end``).
    """

    def __init__(self, blocks: torch.Tensor | None = None, prec="fp64", stream=None,
                 _handle=None, _dims=None):
        self._lib = load_library()
        self.prec = PREC_BY_NAME[prec] if isinstance(prec, str) else int(prec)
        self._h = None
        if _handle is not None:
            self._h = _handle
            self.Nt, self.Nd, self.Nm = _dims
        else:
            blocks = _dev_f64(blocks, "blocks")
            if blocks.dim() != 3:
                raise ValueError("blocks must be [Nt][Nd][Nm]")
            self.Nt, self.Nd, self.Nm = (int(v) for v in blocks.shape)
            h = _vp()
            _check("p2o_setup", self._lib.p2o_setup(
                blocks.data_ptr(), self.Nd, self.Nm, self.Nt, self.prec,
                _stream_handle(stream), _c.byref(h)))
            self._h = h
        L = _i64(0)
        _check("p2o_get_info", self._lib.p2o_get_info(self._h, None, None, None,
                                                      _c.byref(L), None))
        self.L = L.value

    @classmethod
    def begin(cls, Nd: int, Nm: int, Nt: int, prec="fp64", stream=None) -> "Plan":
        lib = load_library()
        p = PREC_BY_NAME[prec] if isinstance(prec, str) else int(prec)
        h = _vp()
        _check("p2o_setup_begin", lib.p2o_setup_begin(Nd, Nm, Nt, p,
                                                      _stream_handle(stream), _c.byref(h)))
        return cls(prec=p, _handle=h, _dims=(Nt, Nd, Nm))

    def setup_columns(self, chunk: torch.Tensor, p0: int, p1: int, stream=None) -> None:
        chunk = _dev_f64(chunk, "chunk")
        if tuple(chunk.shape) != (self.Nt, self.Nd, p1 - p0):
            raise ValueError(f"chunk must be [{self.Nt}][{self.Nd}][{p1 - p0}]")
        _check("p2o_setup_columns", self._lib.p2o_setup_columns(
            self._handle(), chunk.data_ptr(), p0, p1, _stream_handle(stream)))

    def setup_end(self, stream=None) -> None:
        _check("p2o_setup_end", self._lib.p2o_setup_end(self._handle(), _stream_handle(stream)))

    def _handle(self):
        if self._h is None:
            raise RuntimeError("plan has been closed")
        return self._h

    @property
    def handle(self) -> int:
        return self._handle().value

    def reserve(self, nrhs: int, stream=None) -> None:
        _check("p2o_reserve", self._lib.p2o_reserve(self._handle(), nrhs, _stream_handle(stream)))

    def apply(self, op: int, x: torch.Tensor, out: torch.Tensor | None = None,
              stream=None) -> torch.Tensor:
        """y = F x (op=OP_F) or y = F* x (op=OP_FADJ).  x: [Nt][n] or [nrhs][Nt][n]."""
        x = _dev_f64(x, "x")
        n_in, n_out = (self.Nm, self.Nd) if op == OP_F else (self.Nd, self.Nm)
        if x.shape[-2:] != (self.Nt, n_in) or x.dim() not in (2, 3):
            raise ValueError(f"x must end in ({self.Nt}, {n_in}), got {tuple(x.shape)}")
        nrhs = 1 if x.dim() == 2 else int(x.shape[0])
        shape = x.shape[:-1] + (n_out,)
        if out is None:
            out = torch.empty(shape, dtype=torch.float64, device=x.device)
        else:
            out = _dev_f64(out, "out")
            if tuple(out.shape) != tuple(shape):
                raise ValueError(f"out must be {tuple(shape)}")
        _check("p2o_apply", self._lib.p2o_apply(self._handle(), op, x.data_ptr(),
                                                out.data_ptr(), nrhs, _stream_handle(stream)))
        return out

    def F(self, m: torch.Tensor, out=None, stream=None) -> torch.Tensor:
        return self.apply(OP_F, m, out, stream)

    def FT(self, d: torch.Tensor, out=None, stream=None) -> torch.Tensor:
        return self.apply(OP_FADJ, d, out, stream)

    def set_assembly(self, method: str) -> None:
        """How hessian() and qoi_precompute() form their F Gamma_prior F*
        products: "matvec" (one FFT-based product per unit vector, the
        paper's Phase 2; the default) or "gram" (Gram matrix of the
        time-domain blocks, then prefix sums along the block diagonals)."""
        if method not in ASSEMBLY:
            raise ValueError(f"method must be one of {sorted(ASSEMBLY)}")
        _check("p2o_set_assembly", self._lib.p2o_set_assembly(self._handle(), ASSEMBLY[method]))

    def hessian(self, prior_var: float, noise_var: torch.Tensor,
                out: torch.Tensor | None = None, stream=None,
                method: str | None = None) -> torch.Tensor:
        """K = Gamma_noise + F Gamma_prior F*, [(Nt Nd)][(Nt Nd)] float64,
        Gamma_prior = prior_var (I (x) C).  `method`, when given, is set as the
        plan's assembly method first (see set_assembly)."""
        if method is not None:
            self.set_assembly(method)
        n = self.Nt * self.Nd
        noise_var = _dev_f64(noise_var, "noise_var")
        if noise_var.numel() != n:
            raise ValueError(f"noise_var must have {n} entries")
        if out is None:
            out = torch.empty((n, n), dtype=torch.float64, device=noise_var.device)
        else:
            out = _dev_f64(out, "out")
        _check("p2o_hessian_assemble", self._lib.p2o_hessian_assemble(
            self._handle(), float(prior_var), noise_var.data_ptr(), out.data_ptr(),
            _stream_handle(stream)))
        return out

    def posterior(self, K: torch.Tensor, d: torch.Tensor, prior_var: float,
                  refine_steps: int = 1, out=None, stream=None) -> torch.Tensor:
        """m = prior_var F* K^{-1} d; K is overwritten by its Cholesky factor."""
        K = _dev_f64(K, "K")
        d = _dev_f64(d, "d")
        nrhs = 1 if d.dim() == 2 else int(d.shape[0])
        if d.shape[-2:] != (self.Nt, self.Nd):
            raise ValueError("d must end in (Nt, Nd)")
        if out is None:
            out = torch.empty(d.shape[:-1] + (self.Nm,), dtype=torch.float64, device=d.device)
        piv = _i64(-1)
        st = self._lib.p2o_posterior_solve(self._handle(), K.data_ptr(), d.data_ptr(),
                                           out.data_ptr(), nrhs, float(prior_var),
                                           int(refine_steps), _c.byref(piv),
                                           _stream_handle(stream))
        if st == 4:
            err = P2OError("p2o_posterior_solve", st)
            err.failed_pivot = piv.value
            raise err
        _check("p2o_posterior_solve", st)
        return out

    def posterior_mean(self, Kfac: torch.Tensor, d: torch.Tensor, prior_var: float,
                       out=None, stream=None) -> torch.Tensor:
        """Phase 4 online: m = Gamma_prior F* K^{-1} d from the factor left in
        Kfac's lower triangle by posterior() (K is not modified)."""
        Kfac = _dev_f64(Kfac, "Kfac")
        d = _dev_f64(d, "d")
        nrhs = 1 if d.dim() == 2 else int(d.shape[0])
        if d.shape[-2:] != (self.Nt, self.Nd):
            raise ValueError("d must end in (Nt, Nd)")
        n = self.Nt * self.Nd
        if tuple(Kfac.shape) != (n, n):
            raise ValueError(f"Kfac must be ({n}, {n})")
        if out is None:
            out = torch.empty(d.shape[:-1] + (self.Nm,), dtype=torch.float64, device=d.device)
        _check("p2o_posterior_mean", self._lib.p2o_posterior_mean(
            self._handle(), Kfac.data_ptr(), d.data_ptr(), out.data_ptr(), nrhs,
            float(prior_var), _stream_handle(stream)))
        return out

    def posterior_invert(self, Kfac: torch.Tensor, out=None, stream=None) -> torch.Tensor:
        """Offline: K^{-1} (exactly symmetric) from the factor left in Kfac's
        lower triangle by posterior()."""
        Kfac = _dev_f64(Kfac, "Kfac")
        n = self.Nt * self.Nd
        if tuple(Kfac.shape) != (n, n):
            raise ValueError(f"Kfac must be ({n}, {n})")
        if out is None:
            out = torch.empty((n, n), dtype=torch.float64, device=Kfac.device)
        else:
            out = _dev_f64(out, "out")
        _check("p2o_posterior_invert", self._lib.p2o_posterior_invert(
            self._handle(), Kfac.data_ptr(), out.data_ptr(), _stream_handle(stream)))
        return out

    def _kinv_args(self, Kinv, d, out):
        Kinv = _dev_f64(Kinv, "Kinv")
        d = _dev_f64(d, "d")
        nrhs = 1 if d.dim() == 2 else int(d.shape[0])
        if d.shape[-2:] != (self.Nt, self.Nd):
            raise ValueError("d must end in (Nt, Nd)")
        n = self.Nt * self.Nd
        if tuple(Kinv.shape) != (n, n):
            raise ValueError(f"Kinv must be ({n}, {n})")
        if out is None:
            out = torch.empty(d.shape[:-1] + (self.Nm,), dtype=torch.float64, device=d.device)
        return Kinv, d, out, nrhs

    def posterior_mean_kinv(self, Kinv: torch.Tensor, d: torch.Tensor, prior_var: float,
                            out=None, stream=None) -> torch.Tensor:
        """Phase 4 online: m = Gamma_prior F* (K^{-1} d) from posterior_invert()'s
        K^{-1} (stream-ordered)."""
        Kinv, d, out, nrhs = self._kinv_args(Kinv, d, out)
        _check("p2o_posterior_mean_kinv", self._lib.p2o_posterior_mean_kinv(
            self._handle(), Kinv.data_ptr(), d.data_ptr(), out.data_ptr(), nrhs,
            float(prior_var), _stream_handle(stream)))
        return out

    def posterior_mean_kinv_noalloc(self, Kinv: torch.Tensor, d: torch.Tensor, prior_var: float,
                                    out: torch.Tensor = None, stream=None) -> torch.Tensor:
        """As posterior_mean_kinv, on the library's fixed device scratch (no
        device allocation inside the call; pass `out` to allocate nothing at
        all)."""
        Kinv, d, out, nrhs = self._kinv_args(Kinv, d, out)
        _check("p2o_posterior_mean_kinv_noalloc", self._lib.p2o_posterior_mean_kinv_noalloc(
            self._handle(), Kinv.data_ptr(), d.data_ptr(), out.data_ptr(), nrhs,
            float(prior_var), _stream_handle(stream)))
        return out

    def set_prior(self, grid=None, radius: int = 2, length: float = 1.0, delta: float = 0.1,
                  stream=None) -> None:
        """Spatial prior covariance C for the inversion calls
        (Gamma_prior = prior_var (I (x) C)): grid = (nx, ny) with nx * ny = Nm,
        C x = delta x + B B x with B the Gaussian window of half-width
        `radius` and length scale `length`; grid=None restores C = I."""
        if grid is None:
            _check("p2o_set_prior", self._lib.p2o_set_prior(self._handle(), None,
                                                          _stream_handle(stream)))
            return
        pg = _PriorGrid(int(grid[0]), int(grid[1]), int(radius), float(length), float(delta))
        _check("p2o_set_prior", self._lib.p2o_set_prior(self._handle(), _c.byref(pg),
                                                      _stream_handle(stream)))

    def qoi_precompute(self, qoi_plan: "Plan", K: torch.Tensor, prior_var: float,
                       stream=None, method: str | None = None):
        """Phase 3 with this plan as the p2o map and `qoi_plan` as the p2q map:
        (Q, Gq) with Q = Fq Gp F* K^{-1} ([(Nt Nq)][(Nt Nd)]) and
        Gq = Fq Gamma_post Fq* ([(Nt Nq)]^2).  K: as left by posterior().
        `method`, when given, is set as this plan's assembly method first."""
        if method is not None:
            self.set_assembly(method)
        K = _dev_f64(K, "K")
        n, nq = self.Nt * self.Nd, qoi_plan.Nt * qoi_plan.Nd
        if tuple(K.shape) != (n, n):
            raise ValueError(f"K must be ({n}, {n})")
        Q = torch.empty((nq, n), dtype=torch.float64, device=K.device)
        G = torch.empty((nq, nq), dtype=torch.float64, device=K.device)
        _check("p2o_qoi_precompute", self._lib.p2o_qoi_precompute(
            self._handle(), qoi_plan._handle(), K.data_ptr(), float(prior_var), Q.data_ptr(),
            G.data_ptr(), _stream_handle(stream)))
        return Q, G

    def autotune(self, op: int, reps: int = 3, stream=None):
        """Time every candidate product kernel for `op`; keep the fastest.
        Returns (chosen index, per-candidate ms list, -1 = not valid)."""
        n = self.config(op)[1]
        times = (_dbl * n)()
        chosen = _i64(-1)
        _check("p2o_autotune", self._lib.p2o_autotune(self._handle(), op, reps, times, n,
                                                      _c.byref(chosen), _stream_handle(stream)))
        return chosen.value, list(times)

    def config(self, op: int):
        """(current candidate index, number of candidates) for `op`."""
        cfg, n = _i64(0), _i64(0)
        _check("p2o_get_config", self._lib.p2o_get_config(self._handle(), op, _c.byref(cfg),
                                                          _c.byref(n)))
        return cfg.value, n.value

    def set_config(self, op: int, cfg: int) -> None:
        _check("p2o_set_config", self._lib.p2o_set_config(self._handle(), op, cfg))

    def set_mfma_threshold(self, op: int, min_rhs: int) -> None:
        """Use the matrix-core kernels from `min_rhs` right-hand sides on (<= 0: never)."""
        _check("p2o_set_mfma_threshold",
               self._lib.p2o_set_mfma_threshold(self._handle(), op, min_rhs))

    def set_kernel_timing(self, enable: bool) -> None:
        _check("p2o_set_kernel_timing", self._lib.p2o_set_kernel_timing(self._handle(), int(enable)))

    def kernel_time(self, op: int):
        """(total ms, launches) of the block-product kernel since the last read."""
        ms, n = _dbl(0), _i64(0)
        _check("p2o_kernel_time", self._lib.p2o_kernel_time(self._handle(), op,
                                                            _c.byref(ms), _c.byref(n)))
        return ms.value, n.value

    def close(self) -> None:
        if self._h is not None:
            self._lib.p2o_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()


def qoi_predict(Q: torch.Tensor, d: torch.Tensor, stream=None) -> torch.Tensor:
    """Phase 4 QoI prediction q = Q d.  Q: [nq][n]; d: [n] or [nrhs][...]
    with n entries per right-hand side.  Returns [nq] or [nrhs][nq]."""
    Q = _dev_f64(Q, "Q")
    d = _dev_f64(d, "d")
    nq, n = (int(v) for v in Q.shape)
    single = d.numel() == n
    nrhs = 1 if single else int(d.shape[0])
    if d.numel() != nrhs * n:
        raise ValueError(f"d must hold {n} entries per right-hand side")
    q = torch.empty((nrhs, nq), dtype=torch.float64, device=Q.device)
    _check("p2o_qoi_predict", load_library().p2o_qoi_predict(
        Q.data_ptr(), nq, n, d.data_ptr(), q.data_ptr(), nrhs, _stream_handle(stream)))
    return q[0] if single else q


def read_bandwidth(buf: torch.Tensor, sink: torch.Tensor, stream=None) -> None:
    """Enqueue one streaming read of all of `buf` (a device tensor whose byte
    size is a multiple of 16): the device's streaming-read ceiling, timed by
    the caller.  `sink`: a device float64 tensor of at least one entry."""
    if not buf.is_cuda or not sink.is_cuda or sink.dtype != torch.float64:
        raise ValueError("buf and sink must be device tensors, sink float64")
    nbytes = buf.numel() * buf.element_size()
    _check("p2o_read_bandwidth", load_library().p2o_read_bandwidth(
        buf.data_ptr(), nbytes, sink.data_ptr(), _stream_handle(stream)))


class Batch:
    """Independent plans of uneven shape applied together: one persistent
    product launch per apply, optionally captured once into a HIP graph."""

    def __init__(self, plans):
        self._lib = load_library()
        self.plans = list(plans)
        hs = (_vp * len(self.plans))(*[p.handle for p in self.plans])
        h = _vp()
        _check("p2o_batch_create", self._lib.p2o_batch_create(hs, len(self.plans), _c.byref(h)))
        self._h = h

    def _args(self, op, xs, ys):
        if len(xs) != len(self.plans):
            raise ValueError("one input per plan")
        outs, nr = [], []
        for p, x, y in zip(self.plans, xs, ys if ys is not None else [None] * len(xs)):
            x = _dev_f64(x, "x")
            n_in, n_out = (p.Nm, p.Nd) if op == OP_F else (p.Nd, p.Nm)
            if x.shape[-2:] != (p.Nt, n_in) or x.dim() not in (2, 3):
                raise ValueError(f"input must end in ({p.Nt}, {n_in})")
            shape = x.shape[:-1] + (n_out,)
            y = torch.empty(shape, dtype=torch.float64, device=x.device) if y is None else y
            outs.append(_dev_f64(y, "y"))
            nr.append(1 if x.dim() == 2 else int(x.shape[0]))
        n = len(xs)
        return (outs, (_vp * n)(*[t.data_ptr() for t in xs]),
                (_vp * n)(*[t.data_ptr() for t in outs]), (_i64 * n)(*nr))

    def apply(self, op: int, xs, ys=None, stream=None):
        outs, xp, yp, nr = self._args(op, xs, ys)
        _check("p2o_batch_apply", self._lib.p2o_batch_apply(self._h, op, xp, yp, nr,
                                                            _stream_handle(stream)))
        return outs

    def autotune(self, op: int, xs, ys=None, reps: int = 2, stream=None):
        """Time every configuration of the persistent kernel on these inputs
        and keep the fastest.  Returns (chosen, per-candidate ms)."""
        outs, xp, yp, nr = self._args(op, xs, ys)
        n = self.config(op)[1]
        times = (_dbl * n)()
        chosen = _i64(-1)
        _check("p2o_batch_autotune", self._lib.p2o_batch_autotune(
            self._h, op, xp, yp, nr, reps, times, n, _c.byref(chosen), _stream_handle(stream)))
        return chosen.value, list(times)

    def config(self, op: int):
        """(configuration set for op or -1, number of candidates)."""
        c, n = _i64(0), _i64(0)
        _check("p2o_batch_get_config", self._lib.p2o_batch_get_config(self._h, op, _c.byref(c),
                                                                      _c.byref(n)))
        return c.value, n.value

    def set_config(self, op: int, cfg: int) -> None:
        _check("p2o_batch_set_config", self._lib.p2o_batch_set_config(self._h, op, cfg))

    def capture(self, op: int, xs, ys, stream=None) -> "Graph":
        """Graph of one batched apply reading xs and writing ys (fixed buffers)."""
        outs, xp, yp, nr = self._args(op, xs, ys)
        g = _vp()
        _check("p2o_graph_capture", self._lib.p2o_graph_capture(self._h, op, xp, yp, nr,
                                                                _stream_handle(stream), _c.byref(g)))
        return Graph(self._lib, g)

    def close(self):
        if self._h is not None:
            self._lib.p2o_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Graph:
    def __init__(self, lib, h):
        self._lib, self._h = lib, h

    def launch(self, stream=None):
        _check("p2o_graph_launch", self._lib.p2o_graph_launch(self._h, _stream_handle(stream)))

    def close(self):
        if self._h is not None:
            self._lib.p2o_graph_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class P2OApply(torch.autograd.Function):
    """d = F m with the adjoint as the backward: grad_m = F*(grad_d)."""

    @staticmethod
    def forward(ctx, plan: Plan, m: torch.Tensor) -> torch.Tensor:
        ctx.plan = plan
        return plan.F(m.contiguous())

    @staticmethod
    def backward(ctx, g: torch.Tensor):
        return None, ctx.plan.FT(g.contiguous())


class P2OAdjoint(torch.autograd.Function):
    """m = F* d with F as the backward: grad_d = F(grad_m)."""

    @staticmethod
    def forward(ctx, plan: Plan, d: torch.Tensor) -> torch.Tensor:
        ctx.plan = plan
        return plan.FT(d.contiguous())

    @staticmethod
    def backward(ctx, g: torch.Tensor):
        return None, ctx.plan.F(g.contiguous())
