"""ctypes binding of libchefsi.so (argument marshalling only).

torch is imported first so that the HIP runtime it ships is the one the
library binds to (both carry the soname libamdhip64.so.7).  Tensors must be
float64 CUDA tensors whose rows are contiguous (stride(1) == 1); the row
stride is passed as the leading dimension.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional, Tuple

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
library_path = os.path.join(_HERE, "libchefsi.so")
if not os.path.exists(library_path):
    raise ImportError(f"{library_path} is not built; run paper_1606_03416_amd.build.build()")
lib = ctypes.CDLL(library_path)

F64, F32, BF16, BF16X3 = 0, 1, 2, 3
(OP_BOUNDS, OP_FILTER, OP_ORTHONORMALIZE, OP_RAYLEIGH_RITZ, OP_SWEEP, OP_FILTER_BACKWARD, OP_LOSS_BACKWARD,
 OP_DENSITY, OP_LOSS, OP_RAYLEIGH_RITZ_BACKWARD) = range(10)
ERR_ARG, ERR_HIP, ERR_WORKSPACE, ERR_NOT_PD, ERR_EIG, ERR_NONFINITE, ERR_UNSUPPORTED = range(1, 8)

_vp = ctypes.c_void_p
_i = ctypes.c_int
_i64 = ctypes.c_int64
_d = ctypes.c_double
_sz = ctypes.c_size_t
_dp = ctypes.POINTER(ctypes.c_double)


class Stats(ctypes.Structure):
    _fields_ = [("bounds_ms", _d), ("filter_ms", _d), ("filter_steps_ms", _d),
                ("orthonormalize_ms", _d), ("rayleigh_ritz_ms", _d), ("total_ms", _d),
                ("cholqr_passes", _d), ("cholqr_cond_bound", _d)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


def _sig(name, res, *args):
    f = getattr(lib, name)
    f.restype = res
    f.argtypes = list(args)
    return f


_sig("chefsi_version", ctypes.c_char_p)
_sig("chefsi_last_error", ctypes.c_char_p)
_sig("chefsi_plan_create", _i, ctypes.POINTER(_vp), _i, _i, _i, _i, ctypes.POINTER(ctypes.c_int32))
_sig("chefsi_plan_destroy", None, _vp)
_sig("chefsi_plan_n", _i64, _vp)
_sig("chefsi_plan_h_elems", _i64, _vp)
_sig("chefsi_plan_neighbour", _i, _vp, _i, _i)
_sig("chefsi_plan_block_elems", _i64, _vp)
_sig("chefsi_workspace_bytes", _i, _vp, _i, _i, _i, _i, _i, ctypes.POINTER(_sz))
_sig("chefsi_bounds", _i, _vp, _vp, _vp, _i, _vp, _i, _vp, _dp, _vp, _sz, _vp)
_sig("chefsi_filter", _i, _vp, _vp, _i, _d, _d, _d, _i, _vp, _i64, _vp, _i64, _i, _vp, _sz, _vp)
_sig("chefsi_filter_noalloc", _i, _vp, _vp, _i, _d, _d, _d, _i, _vp, _i64, _vp, _i64, _i, _vp)
_sig("chefsi_orthonormalize", _i, _i64, _i, _vp, _i64, _i, _vp, _vp, _sz, _vp)
_sig("chefsi_orthonormalize_workspace_bytes", _i, _i64, _i, _i, ctypes.POINTER(_sz))
_sig("chefsi_rayleigh_ritz", _i, _vp, _vp, _vp, _i64, _i, _vp, _i64, _vp, _vp, _vp, _vp, _sz, _vp)
_sig("chefsi_sweep", _i, _vp, _vp, _i, _i, _i, _i, _vp, _vp, _i, _vp, _i64, _i, _vp, _vp, _vp,
     ctypes.POINTER(Stats), _vp, _sz, _vp)
_sig("chefsi_loss_backward", _i, _vp, _vp, _i, _d, _d, _d, _i, _i, _i, _vp, _i64, _i, _vp, _vp, _i64,
     _dp, _vp, _sz, _vp)
_sig("chefsi_backward_workspace_bytes", _i, _vp, _i, _i, _i, _i, _i, ctypes.POINTER(_sz))
_sig("chefsi_loss", _i, _vp, _vp, _i, _d, _d, _d, _i, _i, _vp, _i64, _i, _dp, _vp, _sz, _vp)
_sig("chefsi_orthonormalize_backward", _i, _i64, _i, _vp, _i64, _vp, _vp, _i64, _vp, _i64, _vp, _sz, _vp)
_sig("chefsi_orthonormalize_backward_workspace_bytes", _i, _i64, _i, ctypes.POINTER(_sz))
_sig("chefsi_rayleigh_ritz_backward", _i, _vp, _vp, _vp, _i64, _i, _vp, _vp, _vp, _i64, _vp, _i, _vp, _sz, _vp)
_sig("chefsi_filter_backward", _i, _vp, _vp, _i, _d, _d, _d, _i, _vp, _i64, _vp, _i64, _i, _vp, _vp,
     _i64, _vp, _sz, _vp)
_sig("chefsi_occupations", _i, _i, _vp, _d, _d, _vp, _vp, _vp)
_sig("chefsi_density_blocks", _i, _vp, _vp, _i64, _i, _vp, _vp, _vp, _sz, _vp)
_sig("chefsi_realign", _i, _vp, _i, _vp, _vp, _vp, _i64, _i, _vp, _sz, _vp)
_sig("chefsi_realign_workspace_bytes", _i, _vp, _i, ctypes.POINTER(_sz))


class ChefsiError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"chefsi error {code}: {msg}")
        self.code = code


def _check(rc: int):
    if rc != 0:
        raise ChefsiError(rc, lib.chefsi_last_error().decode(errors="replace"))


def _p(t: Optional[torch.Tensor]):
    return None if t is None else _vp(t.data_ptr())


def _stream():
    return _vp(torch.cuda.current_stream().cuda_stream)


def _on(t: torch.Tensor, device) -> bool:
    return device is None or t.device == device


def _mv(t, name: str, rows: Optional[int] = None, device=None, dtype=torch.float64) -> int:
    """Checks a multivector (rows x ns, contiguous rows) and returns its row
    stride; every check runs before any library call."""
    if (not torch.is_tensor(t) or not t.is_cuda or t.dtype != dtype or t.dim() != 2 or t.stride(1) != 1
            or not _on(t, device)):
        raise ValueError(f"{name} must be a 2-D {dtype} CUDA tensor with contiguous rows"
                         + ("" if device is None else f" on {device}"))
    if rows is not None and t.shape[0] != rows:
        raise ValueError(f"{name} must have {rows} rows, got {t.shape[0]}")
    ld = t.stride(0) if t.shape[0] > 1 else max(t.shape[1], 1)
    if ld < t.shape[1]:
        raise ValueError(f"{name}: rows overlap (row stride {ld} < {t.shape[1]} columns)")
    return ld


def _vec(t, name: str, n: int, device=None):
    if (not torch.is_tensor(t) or not t.is_cuda or t.dtype != torch.float64 or not t.is_contiguous()
            or t.numel() < n or not _on(t, device)):
        raise ValueError(f"{name} must be a contiguous float64 CUDA tensor of >= {n} elements"
                         + ("" if device is None else f" on {device}"))


def _user_ws(ws, device) -> None:
    if (not torch.is_tensor(ws) or not ws.is_cuda or ws.dtype != torch.uint8 or not ws.is_contiguous()
            or not _on(ws, device)):
        raise ValueError("ws must be a contiguous uint8 CUDA tensor" + ("" if device is None else f" on {device}"))


def _workspace(nbytes: int, device) -> torch.Tensor:
    return torch.empty(max(int(nbytes), 256), dtype=torch.uint8, device=device)


class Plan:
    """Element grid + stencil + ALB counts (the structure of H^DG)."""

    def __init__(self, grid, stencil: int, J):
        J = np.ascontiguousarray(np.asarray(J), dtype=np.int32)
        nx, ny, nz = (int(v) for v in grid)
        self.grid, self.stencil, self.J = (nx, ny, nz), int(stencil), J
        self._h = _vp()
        _check(lib.chefsi_plan_create(ctypes.byref(self._h), nx, ny, nz, int(stencil),
                                      J.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))))
        self.N = int(lib.chefsi_plan_n(self._h))
        self.h_elems = int(lib.chefsi_plan_h_elems(self._h))
        self.block_elems = int(lib.chefsi_plan_block_elems(self._h))
        self.device = torch.device("cuda", torch.cuda.current_device())

    def close(self):
        if getattr(self, "_h", None):
            lib.chefsi_plan_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def neighbour(self, K: int, s: int) -> int:
        return int(lib.chefsi_plan_neighbour(self._h, K, s))

    def workspace_bytes(self, op: int, ns: int, dtype: int = F64, passes: int = 2, lanczos_steps: int = 20) -> int:
        out = _sz(0)
        _check(lib.chefsi_workspace_bytes(self._h, op, ns, dtype, passes, lanczos_steps, ctypes.byref(out)))
        return int(out.value)

    def backward_workspace_bytes(self, op: int, m: int, ns: int, passes: int = 2, ckpt_stride: int = 4) -> int:
        out = _sz(0)
        _check(lib.chefsi_backward_workspace_bytes(self._h, op, m, ns, passes, ckpt_stride, ctypes.byref(out)))
        return int(out.value)

    def _check_H(self, H: torch.Tensor):
        if (not torch.is_tensor(H) or not H.is_cuda or H.dtype != torch.float64 or not H.is_contiguous()
                or H.numel() != self.h_elems or H.device != self.device):
            raise ValueError(f"H must be a contiguous float64 CUDA tensor of {self.h_elems} elements on {self.device}")

    # -- Algorithm 1 step 1
    def bounds(self, H, v0, lanczos_steps: int = 20, ritz_prev=None, ns: Optional[int] = None,
               out: Optional[torch.Tensor] = None) -> Tuple[float, float, float]:
        self._check_H(H)
        _vec(v0, "v0", self.N, self.device)
        if ritz_prev is not None:
            ns = ritz_prev.numel()
            _vec(ritz_prev, "ritz_prev", ns, self.device)
        if ns is None:
            raise ValueError("ns is required for first-cycle bounds")
        if out is not None:
            _vec(out, "out", 3, self.device)
        ws = _workspace(self.workspace_bytes(OP_BOUNDS, ns, lanczos_steps=lanczos_steps), H.device)
        hb = (ctypes.c_double * 3)()
        _check(lib.chefsi_bounds(self._h, _p(H), _p(v0), lanczos_steps, _p(ritz_prev), ns, _p(out),
                                 hb, _p(ws), ws.numel(), _stream()))
        return float(hb[0]), float(hb[1]), float(hb[2])

    # -- Algorithm 1 step 2
    def filter(self, H, X, m: int, a: float, b: float, a0: float, dtype: int = F64,
               out: Optional[torch.Tensor] = None) -> torch.Tensor:
        self._check_H(H)
        ldx = _mv(X, "X", self.N, self.device)
        ns = X.shape[1]
        if out is None:
            out = torch.empty((self.N, ns), dtype=torch.float64, device=X.device)
        ldy = _mv(out, "out", self.N, self.device)
        ws = _workspace(self.workspace_bytes(OP_FILTER, ns, dtype), X.device)
        _check(lib.chefsi_filter(self._h, _p(H), m, a, b, a0, dtype, _p(X), ldx, _p(out), ldy, ns,
                                 _p(ws), ws.numel(), _stream()))
        return out

    def filter_noalloc(self, H, X, m: int, a: float, b: float, a0: float, dtype: int = F64,
                       out: Optional[torch.Tensor] = None) -> torch.Tensor:
        """chefsi_filter without a workspace: the library's static per-GPU
        scratch is used (for callers that cannot allocate; pass `out`)."""
        self._check_H(H)
        ldx = _mv(X, "X", self.N, self.device)
        ns = X.shape[1]
        if out is None:
            out = torch.empty((self.N, ns), dtype=torch.float64, device=X.device)
        ldy = _mv(out, "out", self.N, self.device)
        if out.shape[1] != ns:
            raise ValueError("out must have as many columns as X")
        _check(lib.chefsi_filter_noalloc(self._h, _p(H), m, a, b, a0, dtype, _p(X), ldx, _p(out), ldy, ns,
                                         _stream()))
        return out

    # -- Algorithm 1 steps 4-5
    def rayleigh_ritz(self, H, Yhat, out: Optional[torch.Tensor] = None, want_Q: bool = False,
                      want_resid: bool = True):
        self._check_H(H)
        ldy = _mv(Yhat, "Yhat", self.N, self.device)
        ns = Yhat.shape[1]
        dev = Yhat.device
        if out is None:
            out = torch.empty((self.N, ns), dtype=torch.float64, device=dev)
        ldx = _mv(out, "out", self.N, self.device)
        ritz = torch.empty(ns, dtype=torch.float64, device=dev)
        resid = torch.empty(ns, dtype=torch.float64, device=dev) if want_resid else None
        Q = torch.empty((ns, ns), dtype=torch.float64, device=dev) if want_Q else None
        ws = _workspace(self.workspace_bytes(OP_RAYLEIGH_RITZ, ns), dev)
        _check(lib.chefsi_rayleigh_ritz(self._h, _p(H), _p(Yhat), ldy, ns, _p(out), ldx, _p(ritz),
                                        _p(resid), _p(Q), _p(ws), ws.numel(), _stream()))
        return out, ritz, resid, Q

    # -- Algorithm 1, one full cycle
    def sweep(self, H, X, m: int, *, dtype: int = F64, passes: int = 2, lanczos_steps: int = 20,
              v0=None, bounds=None, ritz=None, warm: bool = False, want_resid: bool = True,
              stats: bool = False, ws: Optional[torch.Tensor] = None):
        """X is updated in place; returns (ritz, resid, bounds_used, stats_dict|None).

        warm=True takes a and a0 from `ritz` (the previous cycle's Ritz values),
        which must then be given.  Every argument is checked here before the
        library is called."""
        self._check_H(H)
        ldx = _mv(X, "X", self.N, self.device)
        ns = X.shape[1]
        dev = X.device
        if v0 is not None:
            _vec(v0, "v0", self.N, self.device)
        elif bounds is None:
            raise ValueError("v0 is required when no bounds are given")
        if ritz is None:
            if warm:
                raise ValueError("warm=True needs the previous Ritz values in `ritz`")
            ritz = torch.empty(ns, dtype=torch.float64, device=dev)
        else:
            _vec(ritz, "ritz", ns, self.device)
        if bounds is not None:
            if not torch.is_tensor(bounds):
                bounds = torch.tensor([float(v) for v in bounds], dtype=torch.float64, device=dev)
            _vec(bounds, "bounds", 3, self.device)
        if ws is not None:
            _user_ws(ws, self.device)
        resid = torch.empty(ns, dtype=torch.float64, device=dev) if want_resid else None
        bout = torch.empty(3, dtype=torch.float64, device=dev)
        need = self.workspace_bytes(OP_SWEEP, ns, dtype, passes, lanczos_steps)
        if ws is None or ws.numel() < need:
            ws = _workspace(need, dev)
        st = Stats()
        _check(lib.chefsi_sweep(self._h, _p(H), m, dtype, passes, lanczos_steps, _p(v0), _p(bounds),
                                1 if warm else 0, _p(X), ldx, ns, _p(ritz), _p(resid), _p(bout),
                                ctypes.byref(st) if stats else None, _p(ws), ws.numel(), _stream()))
        return ritz, resid, bout, (st.as_dict() if stats else None)

    # -- loss of one filter + Cholesky-QR + Rayleigh-Ritz pass (forward only)
    def loss(self, H, X, m: int, a: float, b: float, a0: float, k: int, passes: int = 2) -> float:
        self._check_H(H)
        ldx = _mv(X, "X", self.N, self.device)
        ns = X.shape[1]
        ws = _workspace(self.backward_workspace_bytes(OP_LOSS, m, ns, passes, 1), X.device)
        loss = ctypes.c_double(0.0)
        _check(lib.chefsi_loss(self._h, _p(H), m, a, b, a0, passes, k, _p(X), ldx, ns, ctypes.byref(loss),
                               _p(ws), ws.numel(), _stream()))
        return float(loss.value)

    # -- adjoint of the Ritz values of chefsi_rayleigh_ritz
    def rayleigh_ritz_backward(self, H, Yhat, Q, ritz_bar, Hbar: Optional[torch.Tensor] = None,
                               accumulate: bool = False, out: Optional[torch.Tensor] = None):
        """(Yhat_bar, Hbar) for the cotangent ritz_bar of the Ritz values."""
        self._check_H(H)
        ldy = _mv(Yhat, "Yhat", self.N, self.device)
        ns = Yhat.shape[1]
        _mv(Q, "Q", ns, self.device)
        if Q.shape[1] != ns or not Q.is_contiguous():
            raise ValueError("Q must be a contiguous ns x ns tensor")
        _vec(ritz_bar, "ritz_bar", ns, self.device)
        if Hbar is None:
            if accumulate:
                raise ValueError("accumulate=True needs Hbar")
            Hbar = torch.empty_like(H)
        else:
            self._check_H(Hbar)
        if out is None:
            out = torch.empty((self.N, ns), dtype=torch.float64, device=Yhat.device)
        ldo = _mv(out, "out", self.N, self.device)
        if out.shape[1] != ns:
            raise ValueError("out must have ns columns")
        ws = _workspace(self.workspace_bytes(OP_RAYLEIGH_RITZ_BACKWARD, ns), Yhat.device)
        _check(lib.chefsi_rayleigh_ritz_backward(self._h, _p(H), _p(Yhat), ldy, ns, _p(Q), _p(ritz_bar), _p(out),
                                                 ldo, _p(Hbar), 1 if accumulate else 0, _p(ws), ws.numel(),
                                                 _stream()))
        return out, Hbar

    # -- adjoint of one filter + Cholesky-QR + Rayleigh-Ritz pass
    def loss_backward(self, H, X, m: int, a: float, b: float, a0: float, k: int, passes: int = 2,
                      ckpt_stride: int = 4):
        self._check_H(H)
        ldx = _mv(X, "X", self.N, self.device)
        ns = X.shape[1]
        dev = X.device
        Hbar = torch.empty_like(H)
        Xbar = torch.empty((self.N, ns), dtype=torch.float64, device=dev)
        ws = _workspace(self.backward_workspace_bytes(OP_LOSS_BACKWARD, m, ns, passes, ckpt_stride), dev)
        loss = ctypes.c_double(0.0)
        _check(lib.chefsi_loss_backward(self._h, _p(H), m, a, b, a0, passes, k, ckpt_stride, _p(X), ldx,
                                        ns, _p(Hbar), _p(Xbar), Xbar.stride(0), ctypes.byref(loss),
                                        _p(ws), ws.numel(), _stream()))
        return float(loss.value), Hbar, Xbar

    def filter_backward(self, H, X, Ybar, m: int, a: float, b: float, a0: float, ckpt_stride: int = 4,
                        Hbar: Optional[torch.Tensor] = None):
        self._check_H(H)
        ldx = _mv(X, "X", self.N, self.device)
        ldyb = _mv(Ybar, "Ybar", self.N, self.device)
        ns = X.shape[1]
        if Ybar.shape[1] != ns:
            raise ValueError("Ybar must have as many columns as X")
        dev = X.device
        if Hbar is None:
            Hbar = torch.zeros_like(H)
        else:
            self._check_H(Hbar)
        Xbar = torch.empty((self.N, ns), dtype=torch.float64, device=dev)
        ws = _workspace(self.backward_workspace_bytes(OP_FILTER_BACKWARD, m, ns, 2, ckpt_stride), dev)
        _check(lib.chefsi_filter_backward(self._h, _p(H), m, a, b, a0, ckpt_stride, _p(X), ldx, _p(Ybar),
                                          ldyb, ns, _p(Hbar), _p(Xbar), Xbar.stride(0), _p(ws), ws.numel(),
                                          _stream()))
        return Hbar, Xbar

    # -- after the cycle: diagonal density-matrix blocks (eq. densitymatrix)
    def density_blocks(self, X, f, out: Optional[torch.Tensor] = None, ws: Optional[torch.Tensor] = None):
        """P_KK = X_K diag(f) X_K^T for every element, back to back (flat)."""
        ldx = _mv(X, "X", self.N, self.device)
        ns = X.shape[1]
        _vec(f, "f", ns, self.device)
        if out is None:
            out = torch.empty(self.block_elems, dtype=torch.float64, device=X.device)
        _vec(out, "out", self.block_elems, self.device)
        if ws is not None:
            _user_ws(ws, self.device)
        need = self.workspace_bytes(OP_DENSITY, ns)
        if ws is None or ws.numel() < need:
            ws = _workspace(need, X.device)
        _check(lib.chefsi_density_blocks(self._h, _p(X), ldx, ns, _p(f), _p(out), _p(ws), ws.numel(), _stream()))
        return out

    def split_blocks(self, P: torch.Tensor):
        """Views J_K x J_K of a flat set of element blocks."""
        out, pos = [], 0
        for n in self.J.tolist():
            out.append(P[pos:pos + n * n].view(n, n))
            pos += n * n
        return out

    # -- before the next cycle: re-alignment to a changed basis (eq. basis_rotation_3)
    def realign_workspace_bytes(self, nr: int) -> int:
        out = _sz(0)
        _check(lib.chefsi_realign_workspace_bytes(self._h, nr, ctypes.byref(out)))
        return int(out.value)

    def realign(self, X, V_new, V_old, nr: int, ws: Optional[torch.Tensor] = None):
        """X_K <- V_new,K^T V_old,K X_K in place (V packed element-major as
        V_K^T, J_K rows of nr samples each)."""
        ldx = _mv(X, "X", self.N, self.device)
        ns = X.shape[1]
        _vec(V_new, "V_new", self.N * nr, self.device)
        _vec(V_old, "V_old", self.N * nr, self.device)
        if ws is not None:
            _user_ws(ws, self.device)
        need = self.realign_workspace_bytes(nr)
        if ws is None or ws.numel() < need:
            ws = _workspace(need, X.device)
        _check(lib.chefsi_realign(self._h, nr, _p(V_new), _p(V_old), _p(X), ldx, ns, _p(ws), ws.numel(),
                                  _stream()))
        return X


def occupations(ritz: torch.Tensor, n_occ: float, kT: float, out: Optional[torch.Tensor] = None):
    """Fermi-Dirac occupations and Fermi level of the Ritz values: (f, mu),
    both device tensors (sum f = n_occ)."""
    ns = ritz.numel()
    _vec(ritz, "ritz", ns)
    if out is None:
        out = torch.empty(ns, dtype=torch.float64, device=ritz.device)
    _vec(out, "out", ns)
    mu = torch.empty(1, dtype=torch.float64, device=ritz.device)
    _check(lib.chefsi_occupations(ns, _p(ritz), float(n_occ), float(kT), _p(out), _p(mu), _stream()))
    return out, mu


class ChefsiLoss(torch.autograd.Function):
    """L = sum of the k lowest Ritz values after one filter + Cholesky-QR +
    Rayleigh-Ritz pass (forward: chefsi_loss), with the hand-written adjoint
    (chefsi_loss_backward, which recomputes the forward from checkpoints) as
    its backward.  Bounds are held constant."""

    @staticmethod
    def forward(ctx, H, X, plan, m, bounds, k, passes=2, ckpt_stride=4):
        a, b, a0 = bounds
        ctx.plan, ctx.args = plan, (m, a, b, a0, k, passes, ckpt_stride)
        ctx.save_for_backward(H, X)
        loss = plan.loss(H, X, m, a, b, a0, k, passes)
        return torch.tensor(loss, dtype=torch.float64, device=H.device)

    @staticmethod
    def backward(ctx, g):
        H, X = ctx.saved_tensors
        m, a, b, a0, k, passes, cs = ctx.args
        _, Hbar, Xbar = ctx.plan.loss_backward(H, X, m, a, b, a0, k, passes, cs)
        return g * Hbar, g * Xbar, None, None, None, None, None, None


class ChebFilter(torch.autograd.Function):
    """Y = p_m(H) X (FP64) with the reverse three-term sweep as its backward
    (chefsi_filter_backward, checkpoints every ckpt_stride steps)."""

    @staticmethod
    def forward(ctx, H, X, plan, m, a, b, a0, ckpt_stride=4):
        ctx.plan, ctx.args = plan, (m, a, b, a0, ckpt_stride)
        ctx.save_for_backward(H, X)
        return plan.filter(H, X, m, a, b, a0)

    @staticmethod
    def backward(ctx, Ybar):
        H, X = ctx.saved_tensors
        m, a, b, a0, cs = ctx.args
        Hbar, Xbar = ctx.plan.filter_backward(H, X, Ybar.contiguous(), m, a, b, a0, cs)
        return Hbar, Xbar, None, None, None, None, None, None


def orthonormalize(Y: torch.Tensor, passes: int = 2, want_U: bool = False):
    """Cholesky-QR in place on Y (Algorithm 1 step 3); returns U or None."""
    ldy = _mv(Y, "Y")
    n, ns = Y.shape
    dev = Y.device
    U = torch.empty((ns, ns), dtype=torch.float64, device=dev) if want_U else None
    ws = _workspace(_orth_ws_bytes(n, ns, passes), dev)
    _check(lib.chefsi_orthonormalize(n, ns, _p(Y), ldy, passes, _p(U), _p(ws), ws.numel(), _stream()))
    return U


def orthonormalize_backward(Yhat: torch.Tensor, U: torch.Tensor, Yhat_bar: torch.Tensor,
                            out: Optional[torch.Tensor] = None) -> torch.Tensor:
    """dL/dY for Yhat = Y U^{-1} (the factor chefsi_orthonormalize returns),
    given dL/dYhat.  out may be Yhat_bar itself (in place)."""
    ldy = _mv(Yhat, "Yhat")
    n, ns = Yhat.shape
    dev = Yhat.device
    ldg = _mv(Yhat_bar, "Yhat_bar", n, dev)
    _mv(U, "U", ns, dev)
    if U.shape[1] != ns or not U.is_contiguous():
        raise ValueError("U must be a contiguous ns x ns tensor")
    if Yhat_bar.shape[1] != ns:
        raise ValueError("Yhat_bar must have ns columns")
    if out is None:
        out = torch.empty((n, ns), dtype=torch.float64, device=dev)
    ldo = _mv(out, "out", n, dev)
    if out.shape[1] != ns:
        raise ValueError("out must have ns columns")
    nb = _sz(0)
    _check(lib.chefsi_orthonormalize_backward_workspace_bytes(n, ns, ctypes.byref(nb)))
    ws = _workspace(nb.value, dev)
    _check(lib.chefsi_orthonormalize_backward(n, ns, _p(Yhat), ldy, _p(U), _p(Yhat_bar), ldg, _p(out), ldo,
                                              _p(ws), ws.numel(), _stream()))
    return out


def _orth_ws_bytes(n: int, ns: int, passes: int = 2) -> int:
    out = _sz(0)
    _check(lib.chefsi_orthonormalize_workspace_bytes(n, ns, passes, ctypes.byref(out)))
    return int(out.value)
