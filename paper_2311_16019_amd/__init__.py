"""MI355X (gfx950) sketched-and-truncated polynomial block Krylov solver for
``A X + X B = C1 C2^T`` (Palitta, Schweitzer, Simoncini, arXiv 2311.16019, Algorithm 1).

Thin Python binding over the C ABI of ``libskrylov.so`` (``include/skrylov.h``): this module
only marshals arguments.  Every arithmetic step of a solve runs in the library's HIP
kernels; PyTorch provides device memory and the current stream.  There is no CPU
fallback: without the built library or a GPU the calls raise.
"""
from __future__ import annotations

import ctypes
from dataclasses import dataclass, field

import numpy as np

from . import _lib
from ._lib import SkrError

__all__ = ["Operator", "Result", "solve", "adjoint_solve", "true_residual", "pairing_grads",
           "SylvesterPairing", "SkrError", "version"]


def _torch():
    import torch
    return torch


def _stream(stream):
    torch = _torch()
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def _dev_ptr(t, name, shape=None):
    torch = _torch()
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a CUDA (HIP) tensor")
    if t.dtype != torch.float64:
        raise TypeError(f"{name} must be float64")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous (row-major)")
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} has shape {tuple(t.shape)}, expected {tuple(shape)}")
    return ctypes.c_void_p(t.data_ptr())


def version() -> str:
    return _lib.load().skr_version().decode()


def release_cached_memory() -> None:
    """Return the device memory the library keeps for reuse across calls to the HIP runtime."""
    _lib.check(_lib.load().skr_release_cached_memory())


class Operator:
    """A sparse operator ``M (+ diag)`` resident on the GPU (CSR of ``M`` and ``M^T``)."""

    def __init__(self, handle, n, nnz, diag=None):
        self._h = handle
        self.n = n
        self.nnz = nnz
        self._diag = diag  # the current diagonal term: None or a float64 tensor (host or device)

    @classmethod
    def from_csr(cls, indptr, indices, data, diag=None, stream=None):
        lib = _lib.load()
        indptr = np.ascontiguousarray(indptr, dtype=np.int32)
        indices = np.ascontiguousarray(indices, dtype=np.int32)
        data = np.ascontiguousarray(data, dtype=np.float64)
        n = indptr.shape[0] - 1
        nnz = int(indptr[-1])
        if indices.shape[0] < nnz or data.shape[0] < nnz:
            raise ValueError("indices/data shorter than indptr[-1]")
        dptr = None
        if diag is not None:
            diag = np.array(diag, dtype=np.float64)  # a copy: kept as the operator's diagonal state
            if diag.shape != (n,):
                raise ValueError("diag must have length n")
            dptr = diag.ctypes.data_as(ctypes.c_void_p)
        h = ctypes.c_void_p()
        _lib.check(lib.skr_op_create_csr(n, nnz, indptr.ctypes.data_as(ctypes.c_void_p),
                                         indices.ctypes.data_as(ctypes.c_void_p),
                                         data.ctypes.data_as(ctypes.c_void_p), dptr, _stream(stream),
                                         ctypes.byref(h)))
        return cls(h, n, nnz, None if diag is None else _torch().from_numpy(diag))

    @classmethod
    def from_scipy(cls, M, diag=None, stream=None):
        import scipy.sparse as sp
        M = sp.csr_matrix(M)
        return cls.from_csr(M.indptr, M.indices, M.data, diag=diag, stream=stream)

    def set_diag(self, diag, stream=None):
        """Replace the diagonal term by a float64 vector (or remove it with None).

        A host tensor is copied to the device first.  The operator remembers the vector
        (``diag``), so that a caller can restore an earlier state."""
        lib = _lib.load()
        if diag is not None and not diag.is_cuda:
            diag = diag.to("cuda")
        ptr = None if diag is None else _dev_ptr(diag, "diag", (self.n,))
        _lib.check(lib.skr_op_set_diag(self._h, ptr, _stream(stream)))
        self._diag = diag

    @property
    def diag(self):
        """The current diagonal term (None or a float64 tensor)."""
        return self._diag

    def close(self):
        h = getattr(self, "_h", None)
        lib = getattr(_lib, "_lib", None) if _lib is not None else None
        if h is not None and h.value and lib is not None:
            lib.skr_op_destroy(h)
        self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:  # interpreter shutdown
            pass


@dataclass
class Result:
    X1: object
    X2: object
    iters: int
    ell: int
    rho_rel: float
    status: str
    history: list = field(default_factory=list)
    ms_steps: float = 0.0
    ms_proj: float = 0.0
    ms_recover: float = 0.0
    kernels: dict = field(default_factory=dict)  # family -> (launches, total ms), profile=True only
    proj: dict = field(default_factory=dict)     # last projected solve: newton_iters, neg_a, neg_b, resid
    failed_checks: int = 0                       # checks whose projected equation could not be solved


KERNEL_FAMILIES = ("spmm", "dots", "reduce", "update", "sketch", "whiten")  # skr_result_kernel_stats order


def _params(k=2, maxit=200, p=20, s=0, tol=1e-6, seed=0, zeta=8, precision="fp64", recover="stored",
            trunc_tol=None, profile=False, sketch="sparse_sign", orth="euclidean"):
    prm = _lib.Params()
    _lib.check(_lib.load().skr_params_default(ctypes.byref(prm)))
    if trunc_tol is None:  # the factorisation's cutoff at the accuracy of the bulk arithmetic
        trunc_tol = 1e-12 if precision == "fp64" else 1e-8
    prm.k, prm.maxit, prm.p, prm.s, prm.tol = int(k), int(maxit), int(p), int(s), float(tol)
    prm.seed, prm.zeta, prm.trunc_tol = int(seed) & (2**64 - 1), int(zeta), float(trunc_tol)
    prm.precision = {"fp64": _lib.SKR_FP64, "mixed": _lib.SKR_MIXED}[precision]
    prm.recover = {"stored": _lib.SKR_RECOVER_STORED, "two_pass": _lib.SKR_RECOVER_TWO_PASS}[recover]
    prm.sketch = {"sparse_sign": _lib.SKR_SKETCH_SPARSE_SIGN, "srht": _lib.SKR_SKETCH_SRHT,
                  "none": _lib.SKR_SKETCH_NONE}[sketch]
    prm.orth = {"euclidean": _lib.SKR_ORTH_EUCLIDEAN, "sketched": _lib.SKR_ORTH_SKETCHED}[orth]
    # profile: False, True (every kernel family) or one family's name (only its launches)
    prm.profile = (2 + KERNEL_FAMILIES.index(profile)) if isinstance(profile, str) else (1 if profile else 0)
    return prm


def _collect(h, n1, n2, stream):
    torch = _torch()
    lib = _lib.load()
    ell, iters, rho, st = ctypes.c_int64(), ctypes.c_int32(), ctypes.c_double(), ctypes.c_int32()
    _lib.check(lib.skr_result_info(h, ctypes.byref(ell), ctypes.byref(iters), ctypes.byref(rho), ctypes.byref(st)))
    X1 = torch.empty((n1, ell.value), dtype=torch.float64, device="cuda")
    X2 = torch.empty((n2, ell.value), dtype=torch.float64, device="cuda")
    _lib.check(lib.skr_result_copy_factors(h, ctypes.c_void_p(X1.data_ptr()), ctypes.c_void_p(X2.data_ptr()),
                                           _stream(stream)))
    ln = ctypes.c_int32()
    _lib.check(lib.skr_result_history(h, None, None, 0, ctypes.byref(ln)))
    d = (ctypes.c_int32 * max(1, ln.value))()
    rr = (ctypes.c_double * max(1, ln.value))()
    _lib.check(lib.skr_result_history(h, d, rr, ln.value, ctypes.byref(ln)))
    t = [ctypes.c_double() for _ in range(3)]
    _lib.check(lib.skr_result_timing(h, *(ctypes.byref(x) for x in t)))
    kernels = {}
    cnt = ctypes.c_int32()
    _lib.check(lib.skr_result_kernel_stats(h, 0, ctypes.byref(cnt), None, None, None))
    for i in range(cnt.value):
        nm, nl, ms = ctypes.c_char_p(), ctypes.c_int64(), ctypes.c_double()
        _lib.check(lib.skr_result_kernel_stats(h, i, None, ctypes.byref(nm), ctypes.byref(nl), ctypes.byref(ms)))
        if nl.value:
            kernels[nm.value.decode()] = (nl.value, ms.value)
    ni, na, nb, pr = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32(), ctypes.c_double()
    _lib.check(lib.skr_result_proj_stats(h, ctypes.byref(ni), ctypes.byref(na), ctypes.byref(nb), ctypes.byref(pr)))
    fc = ctypes.c_int32()
    _lib.check(lib.skr_result_failed_checks(h, ctypes.byref(fc)))
    return Result(X1=X1, X2=X2, iters=iters.value, ell=ell.value, rho_rel=rho.value,
                  status=_lib.STATUS_NAMES.get(st.value, str(st.value)),
                  history=[(d[i], rr[i]) for i in range(ln.value)],
                  ms_steps=t[0].value, ms_proj=t[1].value, ms_recover=t[2].value, kernels=kernels,
                  proj=dict(newton_iters=ni.value, neg_a=na.value, neg_b=nb.value, resid=pr.value),
                  failed_checks=fc.value)


def _run(entry, A, B, C1, C2, stream, **params):
    lib = _lib.load()
    r = C1.shape[1]
    p1 = _dev_ptr(C1, "C1", (A.n, r))
    p2 = _dev_ptr(C2, "C2", (B.n, r))
    prm = _params(**params)
    h = ctypes.c_void_p()
    code = getattr(lib, entry)(A._h, B._h, p1, p2, r, ctypes.byref(prm), _stream(stream), ctypes.byref(h))
    _lib.check(code)
    try:
        return _collect(h, A.n, B.n, stream)
    finally:
        lib.skr_result_destroy(h)


def solve(A: Operator, B: Operator, C1, C2, stream=None, **params) -> Result:
    """Solve ``A X + X B = C1 C2^T`` (Algorithm 1); returns ``X ~ X1 X2^T`` on the GPU.

    ``params``: k, maxit, p, s, tol, seed, zeta, precision ('fp64' | 'mixed'),
    recover ('stored' | 'two_pass'), trunc_tol (default 1e-12 in FP64, 1e-8 in mixed precision),
    sketch ('sparse_sign': s-PKSM, Algorithm 1;
    'srht': s-PKSM with the subsampled randomized DCT of Sec. 6; 'none': t-PKSM, Algorithm 2,
    no embedding), orth ('euclidean' | 'sketched': truncated
    Gram-Schmidt and QR in the sketched inner product, appendix A).
    """
    return _run("skr_solve", A, B, C1, C2, stream, **params)


def adjoint_solve(A: Operator, B: Operator, G1, G2, stream=None, **params) -> Result:
    """Solve the transposed equation ``A^T L + L B^T = G1 G2^T`` with the same method."""
    return _run("skr_adjoint_solve", A, B, G1, G2, stream, **params)


def lyap_solve(A: Operator, C, stream=None, **params) -> Result:
    """Solve the Lyapunov equation ``A X + X A^T = C C^T`` on one Krylov space (the
    specialisation of Algorithm 1 with ``B = A^T``, ``C2 = C1``); ``X ~ X1 X2^T`` is
    symmetric.  Same ``params`` as :func:`solve` (two-pass block step and stored basis)."""
    lib = _lib.load()
    r = C.shape[1]
    pc = _dev_ptr(C, "C", (A.n, r))
    prm = _params(**params)
    h = ctypes.c_void_p()
    _lib.check(lib.skr_lyap_solve(A._h, pc, r, ctypes.byref(prm), _stream(stream), ctypes.byref(h)))
    try:
        return _collect(h, A.n, A.n, stream)
    finally:
        lib.skr_result_destroy(h)


def true_residual(A: Operator, B: Operator, X1, X2, C1, C2, stream=None, adjoint=False) -> float:
    """``||A X + X B - C1 C2^T||_F / ||C1 C2^T||_F`` for ``X = X1 X2^T`` (on the GPU);
    with ``adjoint=True`` the transposed equation's ``||A^T X + X B^T - C1 C2^T||_F / ||C1 C2^T||_F``."""
    lib = _lib.load()
    ell, r = X1.shape[1], C1.shape[1]
    out = ctypes.c_double()
    entry = lib.skr_true_residual_adjoint if adjoint else lib.skr_true_residual
    _lib.check(entry(A._h, B._h, _dev_ptr(X1, "X1", (A.n, ell)), _dev_ptr(X2, "X2", (B.n, ell)), ell,
                                     _dev_ptr(C1, "C1", (A.n, r)), _dev_ptr(C2, "C2", (B.n, r)), r, _stream(stream),
                                     ctypes.byref(out)))
    return out.value


def pairing_grads(X1, X2, C1, C2, P1, P2, L1=None, L2=None, stream=None, want=("dC1", "dC2", "dsig", "dP1", "dP2")):
    """Loss ``tr(P1^T X1 X2^T P2)`` and its gradients given adjoint factors ``L1 L2^T``."""
    torch = _torch()
    lib = _lib.load()
    n1, ellx = X1.shape
    n2 = X2.shape[0]
    r, q = C1.shape[1], P1.shape[1]
    outs = {}
    shapes = {"dC1": (n1, r), "dC2": (n2, r), "dsig": (n1,), "dP1": (n1, q), "dP2": (n2, q)}
    for key in want:
        outs[key] = torch.empty(shapes[key], dtype=torch.float64, device="cuda")
    ptr = {k: (ctypes.c_void_p(outs[k].data_ptr()) if k in outs else None) for k in shapes}
    elll = 0 if L1 is None else L1.shape[1]
    loss = ctypes.c_double()
    _lib.check(lib.skr_pairing_grads(
        n1, n2, r, q, _dev_ptr(X1, "X1"), _dev_ptr(X2, "X2"), ellx,
        None if L1 is None else _dev_ptr(L1, "L1"), None if L2 is None else _dev_ptr(L2, "L2"), elll,
        _dev_ptr(C1, "C1"), _dev_ptr(C2, "C2"), _dev_ptr(P1, "P1"), _dev_ptr(P2, "P2"), ctypes.byref(loss),
        ptr["dC1"], ptr["dC2"], ptr["dsig"], ptr["dP1"], ptr["dP2"], _stream(stream)))
    outs["loss"] = loss.value
    return outs


def _make_pairing():
    torch = _torch()

    class SylvesterPairing(torch.autograd.Function):
        """``L = tr(P1^T X P2)`` with ``X`` solving ``(A0 + diag(sigma)) X + X B = C1 C2^T``.

        Forward: set ``sigma`` as the diagonal term of ``A0``, solve (Algorithm 1).
        Backward: one adjoint solve ``A^T Lam + Lam B^T = P1 P2^T`` with the same kernels,
        then ``dC1 = Lam C2``, ``dC2 = Lam^T C1``, ``dsigma = -diag(Lam X^T)``,
        ``dP1 = X P2``, ``dP2 = X^T P1`` (all scaled by the incoming gradient).
        ``sigma = None`` solves with ``A0`` itself (no diagonal term).  Each of the two
        solves sets its own ``sigma`` on ``A0`` and restores ``A0``'s previous diagonal
        afterwards, so several forwards may run before their backwards.
        """

        @staticmethod
        def forward(ctx, C1, C2, sigma, P1, P2, A0, B, params):
            params = dict(params or {})
            sig = sigma.detach().clone().contiguous() if sigma is not None else None
            prev = A0.diag
            A0.set_diag(sig)
            try:
                res = solve(A0, B, C1.detach().contiguous(), C2.detach().contiguous(), **params)
            finally:
                A0.set_diag(prev)
            out = pairing_grads(res.X1, res.X2, C1.detach().contiguous(), C2.detach().contiguous(),
                                P1.detach().contiguous(), P2.detach().contiguous(), want=())
            ctx.save_for_backward(C1, C2, P1, P2, res.X1, res.X2)
            ctx.A0, ctx.B, ctx.params, ctx.sigma = A0, B, params, sig
            ctx.fwd = res
            return torch.tensor(out["loss"], dtype=torch.float64, device=C1.device)

        @staticmethod
        def backward(ctx, g):
            C1, C2, P1, P2, X1, X2 = ctx.saved_tensors
            prev = ctx.A0.diag
            ctx.A0.set_diag(ctx.sigma)  # the operator of this forward, whatever ran since
            try:
                adj = adjoint_solve(ctx.A0, ctx.B, P1.detach().contiguous(), P2.detach().contiguous(), **ctx.params)
            finally:
                ctx.A0.set_diag(prev)
            ctx.adj = adj
            gr = pairing_grads(X1, X2, C1.detach().contiguous(), C2.detach().contiguous(), P1.detach().contiguous(),
                               P2.detach().contiguous(), L1=adj.X1, L2=adj.X2)
            gs = g.to(torch.float64)
            dsig = gs * gr["dsig"] if ctx.sigma is not None else None
            return (gs * gr["dC1"], gs * gr["dC2"], dsig, gs * gr["dP1"], gs * gr["dP2"], None, None, None)

    return SylvesterPairing


class _LazyPairing:
    _cls = None

    def __getattr__(self, name):
        if _LazyPairing._cls is None:
            _LazyPairing._cls = _make_pairing()
        return getattr(_LazyPairing._cls, name)


SylvesterPairing = _LazyPairing()
