"""Partition-and-combine maximum-pseudo-likelihood copula estimation on
AMD Instinct MI355X (arXiv:1609.05530), Python binding of libcpc.

Every step runs in the HIP kernels of libcpc.so; this module only moves
arguments: torch tensors supply device memory and the current stream.

    import paper_1609_05530_amd as cpc
    res = cpc.fit(x, y, offsets, "frank", prec="fp32c")   # x, y: cuda tensors
    res.theta, res.var, res.status, res.combined_theta
"""
from __future__ import annotations

import ctypes
import dataclasses
from typing import Dict, Optional, Sequence

import numpy as np
import torch

from ._lib import CpcError, Options, check, lib

FAMILIES = {"gaussian": 0, "frank": 1, "gumbel": 2}
PRECISIONS = {"fp64": 0, "fp32c": 1}
TIES = {"average": 0, "first": 1}
VARIANCES = {"ggr": 0, "invinfo": 1}
STATUS = {0: "OK", 1: "BOUNDARY_NATURAL", 2: "BOUNDARY_BOX", 3: "DEGENERATE", 4: "NONFINITE", 5: "NOCONV",
          6: "BADVAR"}

__all__ = ["fit", "fit_batched", "rank", "eval_subsets", "variance", "LogLik", "Score", "FitResult",
           "CpcError", "workspace_bytes", "sample", "density_distance", "replicate_summary", "spearman_fit",
           "kendall_fit", "rank_margins", "gaussk_fit", "FAMILIES", "STATUS"]


def _code(table, v):
    return table[v] if isinstance(v, str) else int(v)


def _options(prec="fp64", ties="average", var="ggr", max_iter=60, tol=0.0, n_min=2, graph=False,
             phase_times=False, schedule=None) -> Options:
    """schedule: None (the library's default, autotuned rank shapes), 0 (built-in
    shapes) or 1 + a rank shape index (that shape for its size class)."""
    o = Options()
    lib().cpc_default_options(ctypes.byref(o))
    if schedule is not None:
        o.schedule = int(schedule)
    o.prec = _code(PRECISIONS, prec)
    o.ties = _code(TIES, ties)
    o.var = _code(VARIANCES, var)
    o.max_iter = int(max_iter)
    o.tol = float(tol)
    o.n_min = int(n_min)
    o.flags = (1 if graph else 0) | (2 if phase_times else 0)
    return o


def phase_times(device=None):
    """Milliseconds of (rank, fit, variance, combine) of the last fit made with
    phase_times=True on this device (HIP events on the fit's stream)."""
    dev = torch.device("cuda", torch.cuda.current_device() if device is None else device)
    ms = (ctypes.c_float * 4)()
    check(lib().cpc_phase_times(_handle(dev), ms))
    return [float(v) for v in ms]


_handles: Dict[int, ctypes.c_void_p] = {}


def _handle(device: torch.device) -> ctypes.c_void_p:
    idx = device.index if device.index is not None else torch.cuda.current_device()
    h = _handles.get(idx)
    if h is None:
        h = ctypes.c_void_p()
        check(lib().cpc_create(idx, ctypes.byref(h)))
        _handles[idx] = h
    return h


def _i64(a) -> np.ndarray:
    if isinstance(a, torch.Tensor):
        a = a.detach().cpu().numpy()
    return np.ascontiguousarray(a, dtype=np.int64)


def _dev(t: torch.Tensor, name: str) -> torch.Tensor:
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a CUDA (HIP) tensor")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    return t


def _dtype_code(t: torch.Tensor) -> int:
    if t.dtype == torch.float64:
        return 0
    if t.dtype == torch.float32:
        return 1
    raise TypeError(f"x and y must be float32 or float64, got {t.dtype}")


def _stream(device) -> int:
    return torch.cuda.current_stream(device).cuda_stream


def workspace_bytes(n: int, K: int, G: int = 1, dtype=torch.float64, offsets=None, **opt) -> int:
    """Workspace bytes for a call: exact for the partition `offsets` when
    given (cpc_workspace_bytes_for), else the upper bound over all partitions
    of n rows into K subsets (cpc_workspace_bytes)."""
    o = _options(**opt)
    dt = 0 if dtype == torch.float64 else 1
    if offsets is not None:
        off = _i64(offsets)
        return _exact_bytes(off, int(G), dt, o)
    return int(lib().cpc_workspace_bytes(int(n), int(K), int(G), dt, ctypes.byref(o)))


def _exact_bytes(off: np.ndarray, G: int, dt: int, o: Options) -> int:
    nbytes = int(lib().cpc_workspace_bytes_for(off.ctypes.data, off.shape[0] - 1, G, dt, ctypes.byref(o)))
    if nbytes == 0:
        raise ValueError("offsets are not a partition of the rows")
    return nbytes


def _workspace(nbytes: int, device, workspace: Optional[torch.Tensor]) -> torch.Tensor:
    if workspace is not None:
        if workspace.numel() * workspace.element_size() < nbytes:
            raise ValueError(f"workspace holds {workspace.numel() * workspace.element_size()} bytes, need {nbytes}")
        return workspace
    return torch.empty(max(nbytes, 1), dtype=torch.uint8, device=device)


@dataclasses.dataclass
class FitResult:
    """Per-subset and per-group results (device tensors)."""
    raw: torch.Tensor       # (K, 6) float64 view of cpc_subset_result_t
    raw_comb: torch.Tensor  # (G, 5) float64 view of cpc_combined_t

    @property
    def theta(self): return self.raw[:, 0]
    @property
    def var(self): return self.raw[:, 1]
    @property
    def loglik(self): return self.raw[:, 2]
    @property
    def score(self): return self.raw[:, 3]
    @property
    def n(self): return self.raw.view(torch.int64)[:, 4]
    @property
    def iters(self): return self.raw.view(torch.int32)[:, 10]
    @property
    def status(self): return self.raw.view(torch.int32)[:, 11]
    @property
    def combined_theta(self): return self.raw_comb[:, 0]
    @property
    def combined_var(self): return self.raw_comb[:, 1]
    @property
    def n_used(self): return self.raw_comb.view(torch.int64)[:, 2]
    @property
    def n_excluded(self): return self.raw_comb.view(torch.int64)[:, 3]
    @property
    def combined_status(self): return self.raw_comb.view(torch.int32)[:, 8]


def fit(x: torch.Tensor, y: torch.Tensor, offsets, family, *, workspace: Optional[torch.Tensor] = None,
        **opt) -> FitResult:
    """Fit every subset [offsets[m], offsets[m+1]) with one family and combine
    them (eq. 12-15 of arXiv:1609.05530)."""
    offsets = _i64(offsets)
    K = offsets.shape[0] - 1
    return fit_batched(x, y, offsets, np.array([0, K], dtype=np.int64), [family], workspace=workspace, **opt)


def fit_batched(x: torch.Tensor, y: torch.Tensor, offsets, group_offsets, families: Sequence, *,
                workspace: Optional[torch.Tensor] = None, out: Optional[FitResult] = None, **opt) -> FitResult:
    """Batched fit (eq. 16): group g = subsets [group_offsets[g], group_offsets[g+1])
    fitted with families[g] and combined on their own."""
    x = _dev(x, "x")
    y = _dev(y, "y")
    if y.dtype != x.dtype or y.shape != x.shape or x.dim() != 1:
        raise ValueError("x and y must be 1-D tensors of equal length and dtype")
    offsets = _i64(offsets)
    gofs = _i64(group_offsets)
    K = offsets.shape[0] - 1
    G = gofs.shape[0] - 1
    fams = np.ascontiguousarray([_code(FAMILIES, f) for f in families], dtype=np.int32)
    o = _options(**opt)
    dt = _dtype_code(x)
    n = x.shape[0]
    ws = _workspace(_exact_bytes(offsets, G, dt, o), x.device, workspace)
    if out is None:
        out = FitResult(torch.empty((K, 6), dtype=torch.float64, device=x.device),
                        torch.empty((G, 5), dtype=torch.float64, device=x.device))
    check(lib().cpc_fit_batched(
        _handle(x.device), x.data_ptr(), y.data_ptr(), dt, n, offsets.ctypes.data, K, gofs.ctypes.data, G,
        fams.ctypes.data, ctypes.byref(o), ws.data_ptr(), ws.numel() * ws.element_size(), out.raw.data_ptr(),
        out.raw_comb.data_ptr(), _stream(x.device)))
    return out


def rank(x: torch.Tensor, y: torch.Tensor, offsets, *, workspace=None, **opt):
    """Doubled ranks R = 2 r of eq. (12) within each subset (uint32 stored in int32 tensors)."""
    x = _dev(x, "x")
    y = _dev(y, "y")
    offsets = _i64(offsets)
    K = offsets.shape[0] - 1
    o = _options(**opt)
    dt = _dtype_code(x)
    n = x.shape[0]
    ws = _workspace(_exact_bytes(offsets, 1, dt, o), x.device, workspace)
    R1 = torch.empty(n, dtype=torch.int32, device=x.device)
    R2 = torch.empty(n, dtype=torch.int32, device=x.device)
    check(lib().cpc_rank(_handle(x.device), x.data_ptr(), y.data_ptr(), dt, n, offsets.ctypes.data, K,
                         ctypes.byref(o), ws.data_ptr(), ws.numel() * ws.element_size(), R1.data_ptr(), R2.data_ptr(),
                         _stream(x.device)))
    return R1, R2


def eval_subsets(R1: torch.Tensor, R2: torch.Tensor, offsets, family, theta: torch.Tensor, *,
                 workspace=None, **opt) -> torch.Tensor:
    """Per subset (sum l, sum dl/dtheta, sum d2l/dtheta2) at theta (shape (K, 3), float64)."""
    R1 = _dev(R1, "R1")
    R2 = _dev(R2, "R2")
    theta = _dev(theta.to(torch.float64).contiguous(), "theta")
    offsets = _i64(offsets)
    K = offsets.shape[0] - 1
    n = R1.shape[0]
    o = _options(**opt)
    ws = _workspace(_exact_bytes(offsets, 1, 0, o), R1.device, workspace)
    out = torch.empty((K, 3), dtype=torch.float64, device=R1.device)
    check(lib().cpc_eval(_handle(R1.device), R1.data_ptr(), R2.data_ptr(), n, offsets.ctypes.data, K,
                         _code(FAMILIES, family), theta.data_ptr(), ctypes.byref(o), ws.data_ptr(), ws.numel() * ws.element_size(),
                         out.data_ptr(), _stream(R1.device)))
    return out


def variance(R1: torch.Tensor, R2: torch.Tensor, offsets, family, theta: torch.Tensor, *, workspace=None,
             **opt) -> torch.Tensor:
    """Asymptotic variance of each subset estimate at theta (Sec. 2.3)."""
    R1 = _dev(R1, "R1")
    R2 = _dev(R2, "R2")
    theta = _dev(theta.to(torch.float64).contiguous(), "theta")
    offsets = _i64(offsets)
    K = offsets.shape[0] - 1
    n = R1.shape[0]
    o = _options(**opt)
    ws = _workspace(_exact_bytes(offsets, 1, 0, o), R1.device, workspace)
    out = torch.empty(K, dtype=torch.float64, device=R1.device)
    check(lib().cpc_variance(_handle(R1.device), R1.data_ptr(), R2.data_ptr(), n, offsets.ctypes.data, K,
                             _code(FAMILIES, family), theta.data_ptr(), ctypes.byref(o), ws.data_ptr(), ws.numel() * ws.element_size(),
                             out.data_ptr(), _stream(R1.device)))
    return out


class LogLik(torch.autograd.Function):
    """theta (K,) -> per-subset pseudo log-likelihood eq. (13); its gradient is
    the score and the score's gradient the Hessian, all three from one launch
    of the hand-written adjoint kernel (kept for the backward passes)."""

    @staticmethod
    def forward(ctx, theta, R1, R2, offsets, family, prec="fp32c"):
        out = eval_subsets(R1, R2, offsets, family, theta.detach(), prec=prec)
        ctx.save_for_backward(theta, out[:, 1].clone(), out[:, 2].clone())
        return out[:, 0].clone()

    @staticmethod
    def backward(ctx, g):
        theta, score, hess = ctx.saved_tensors
        return g * _Known.apply(theta, score, hess), None, None, None, None, None


class _Known(torch.autograd.Function):
    """theta -> a value already computed at theta, whose derivative with
    respect to theta is also known (the score and its Hessian)."""

    @staticmethod
    def forward(ctx, theta, value, derivative):
        ctx.save_for_backward(derivative)
        return value.clone()

    @staticmethod
    def backward(ctx, g):
        (derivative,) = ctx.saved_tensors
        return g * derivative, None, None


class Score(torch.autograd.Function):
    """theta (K,) -> per-subset score sum dl/dtheta; its gradient is the
    Hessian sum d2l/dtheta2 from the same adjoint kernel (double backward)."""

    @staticmethod
    def forward(ctx, theta, R1, R2, offsets, family, prec="fp32c"):
        out = eval_subsets(R1, R2, offsets, family, theta.detach(), prec=prec)
        ctx.save_for_backward(out[:, 2].clone())
        return out[:, 1].clone()

    @staticmethod
    def backward(ctx, g):
        (hess,) = ctx.saved_tensors
        return g * hess, None, None, None, None, None


# --------------------------------------------------------------------------
# The simulation study of Sec. 2.5-2.6 (inputs drawn on the device, metrics)

def _device(device) -> torch.device:
    if device is None:
        return torch.device("cuda", torch.cuda.current_device())
    d = torch.device(device)
    return torch.device("cuda", d.index if d.index is not None else torch.cuda.current_device())


def sample(family, theta: float, n: int, *, seed: int = 0, row0: int = 0, dtype=torch.float64, device=None):
    """Rows row0 .. row0+n-1 of the seeded stream of pairs with N(0, 1)
    margins and the family's copula at theta (Sec. 2.5), drawn on the GPU."""
    dev = _device(device)
    x = torch.empty(int(n), dtype=dtype, device=dev)
    y = torch.empty(int(n), dtype=dtype, device=dev)
    check(lib().cpc_sample(_handle(dev), _code(FAMILIES, family), float(theta), ctypes.c_uint64(int(seed)),
                           int(row0), int(n), _dtype_code(x), x.data_ptr(), y.data_ptr(), _stream(dev)))
    return x, y


def _theta_vec(t, dev) -> torch.Tensor:
    if isinstance(t, torch.Tensor):
        return t.to(device=dev, dtype=torch.float64).reshape(-1).contiguous()
    return torch.as_tensor(np.atleast_1d(np.asarray(t, dtype=np.float64)), device=dev)


# Normal-score box of the density distances per family: 20 holds the
# squared Gaussian density to 1e-9 up to |rho| = 0.9; the Gumbel density's
# square is not integrable at (1, 1), its integrals grow with the box, and
# over |s|, |t| <= 8.3 (u, v within 1e-16 of the square's edges) the rule
# resolves it.
DISTANCE_BOX = {"gaussian": 20.0, "frank": 20.0, "gumbel": 8.3}


def density_distance(family, theta_a, theta_b, *, panels: int = 256, box: Optional[float] = None,
                     device=None) -> torch.Tensor:
    """(P, 4) tensor per parameter pair: int |c_a - c_b|, int c_a,
    int (c_a - c_b)^2, int c_a^2 over the unit square (eq. 19 = [:, 0] / [:, 1],
    eq. 20 = sqrt([:, 2] / [:, 3])), in normal-score coordinates over
    |s|, |t| <= box (default DISTANCE_BOX[family])."""
    if box is None:
        box = DISTANCE_BOX[family if isinstance(family, str) else [k for k, v in FAMILIES.items() if v == family][0]]
    dev = _device(device if device is not None else (theta_a.device if isinstance(theta_a, torch.Tensor) else None))
    ta = _theta_vec(theta_a, dev)
    tb = _theta_vec(theta_b, dev)
    if ta.numel() != tb.numel():
        raise ValueError("theta_a and theta_b must have the same length")
    P = ta.numel()
    ws = torch.empty(32 * P * int(panels), dtype=torch.uint8, device=dev)
    out = torch.empty((P, 4), dtype=torch.float64, device=dev)
    check(lib().cpc_density_distance(_handle(dev), _code(FAMILIES, family), P, ta.data_ptr(), tb.data_ptr(),
                                     float(box), int(panels), ws.data_ptr(), ws.numel(), out.data_ptr(),
                                     _stream(dev)))
    return out


def replicate_summary(combined: torch.Tensor, full: torch.Tensor) -> torch.Tensor:
    """[eq. 17, eq. 18, bias, MSE, replicates used] from the per-replicate
    combined results (eq. 16) and full-data results ((S, 5) float64 views of
    cpc_combined_t, e.g. FitResult.raw_comb)."""
    combined = _dev(combined.contiguous(), "combined")
    full = _dev(full.contiguous(), "full")
    if combined.shape != full.shape or combined.dim() != 2 or combined.shape[1] != 5:
        raise ValueError("combined and full must be (S, 5) views of cpc_combined_t")
    out = torch.empty(5, dtype=torch.float64, device=combined.device)
    check(lib().cpc_replicate_summary(_handle(combined.device), combined.shape[0], combined.data_ptr(),
                                      full.data_ptr(), out.data_ptr(), _stream(combined.device)))
    return out


PARTITION_SCHEMES = {"contiguous": 0, "blocks": 1, "strided": 2}


def partition(x: torch.Tensor, y: torch.Tensor, rep_offsets, M: int, scheme: str = "contiguous", *,
              workspace: Optional[torch.Tensor] = None):
    """Each replicate (rows rep_offsets[r] .. rep_offsets[r+1] - 1) split into
    M subsets by a partitioning scheme (cpc_partition): "contiguous" (equal
    runs of stored rows), "blocks" (equal runs of the x-order) or "strided"
    (every M-th row of the x-order). Returns (x_out, y_out, offsets) with
    offsets a host int64 array of R M + 1 subset bounds, ready for
    fit_batched with one group of M subsets per replicate."""
    x = _dev(x, "x")
    y = _dev(y, "y")
    if x.shape != y.shape or x.dtype != y.dtype or x.dim() != 1:
        raise ValueError("x and y must be 1-D tensors of one shape and dtype")
    rep = _i64(rep_offsets)
    R = rep.shape[0] - 1
    code = _code(PARTITION_SCHEMES, scheme)
    dt = _dtype_code(x)
    # 0 for arguments the call itself rejects (with the reason)
    need = max(int(lib().cpc_partition_workspace_bytes(rep.ctypes.data, R, dt, code)) if R >= 1 else 0, 1)
    if workspace is None or workspace.numel() < need:
        workspace = torch.empty(need, dtype=torch.uint8, device=x.device)
    xo = torch.empty_like(x)
    yo = torch.empty_like(y)
    # (an M the library rejects gets a placeholder; nothing is written to it)
    offs = np.empty(R * int(M) + 1 if R >= 1 and 1 <= int(M) < 2 ** 31 else 1, dtype=np.int64)
    check(lib().cpc_partition(_handle(x.device), x.data_ptr(), y.data_ptr(), dt, x.shape[0], rep.ctypes.data, R,
                              int(M), code, workspace.data_ptr(), workspace.numel(), xo.data_ptr(), yo.data_ptr(),
                              offs.ctypes.data, _stream(x.device)))
    return xo, yo, offs


def spearman_fit(R1: torch.Tensor, R2: torch.Tensor, offsets, families, group_offsets=None, *, n_min: int = 2,
                 workspace: Optional[torch.Tensor] = None) -> FitResult:
    """The inversion of Spearman's rho per subset from doubled ranks (as made
    by rank()), combined per group by eq. (15). ``families``: one family, or
    one per group."""
    R1 = _dev(R1, "R1")
    R2 = _dev(R2, "R2")
    offsets = _i64(offsets)
    K = offsets.shape[0] - 1
    gofs = _i64(group_offsets if group_offsets is not None else [0, K])
    G = gofs.shape[0] - 1
    if isinstance(families, (str, int)):
        families = [families] * G
    fams = np.ascontiguousarray([_code(FAMILIES, f) for f in families], dtype=np.int32)
    n = R1.shape[0]
    o = _options(n_min=n_min)
    nbytes = int(lib().cpc_spearman_workspace_bytes(n, K, G))
    ws = _workspace(nbytes, R1.device, workspace)
    out = FitResult(torch.empty((K, 6), dtype=torch.float64, device=R1.device),
                    torch.empty((G, 5), dtype=torch.float64, device=R1.device))
    check(lib().cpc_spearman_fit(_handle(R1.device), R1.data_ptr(), R2.data_ptr(), n, offsets.ctypes.data, K,
                                 gofs.ctypes.data, G, fams.ctypes.data, ctypes.byref(o), ws.data_ptr(),
                                 ws.numel() * ws.element_size(), out.raw.data_ptr(), out.raw_comb.data_ptr(),
                                 _stream(R1.device)))
    return out


def kendall_fit(R1: torch.Tensor, R2: torch.Tensor, offsets, families, group_offsets=None, *, n_min: int = 2,
                 workspace: Optional[torch.Tensor] = None) -> FitResult:
    """The inversion of Kendall's tau per subset (at most 2^20 rows) from
    doubled ranks (as made by rank()), combined per group by eq. (15).
    ``families``: one family, or one per group."""
    R1 = _dev(R1, "R1")
    R2 = _dev(R2, "R2")
    offsets = _i64(offsets)
    K = offsets.shape[0] - 1
    gofs = _i64(group_offsets if group_offsets is not None else [0, K])
    G = gofs.shape[0] - 1
    if isinstance(families, (str, int)):
        families = [families] * G
    fams = np.ascontiguousarray([_code(FAMILIES, f) for f in families], dtype=np.int32)
    n = R1.shape[0]
    o = _options(n_min=n_min)
    nbytes = int(lib().cpc_kendall_workspace_bytes(n, K, G))
    ws = _workspace(nbytes, R1.device, workspace)
    out = FitResult(torch.empty((K, 6), dtype=torch.float64, device=R1.device),
                    torch.empty((G, 5), dtype=torch.float64, device=R1.device))
    check(lib().cpc_kendall_fit(_handle(R1.device), R1.data_ptr(), R2.data_ptr(), n, offsets.ctypes.data, K,
                                gofs.ctypes.data, G, fams.ctypes.data, ctypes.byref(o), ws.data_ptr(),
                                ws.numel() * ws.element_size(), out.raw.data_ptr(), out.raw_comb.data_ptr(),
                                _stream(R1.device)))
    return out


def rank_margins(X: torch.Tensor, offsets, **opt) -> torch.Tensor:
    """Doubled ranks (eq. 12) of every margin of X (k x n, one margin per row)
    within each subset: (k, n) int32, two margins per cpc_rank call."""
    X = _dev(X, "X")
    if X.dim() != 2:
        raise ValueError("X must be k x n")
    k = X.shape[0]
    R = torch.empty(X.shape, dtype=torch.int32, device=X.device)
    for j in range(0, k, 2):
        a, b = rank(X[j].contiguous(), X[min(j + 1, k - 1)].contiguous(), offsets, **opt)
        R[j].copy_(a)
        if j + 1 < k:
            R[j + 1].copy_(b)
    return R


def gaussk_fit(R: torch.Tensor, offsets, group_offsets=None, *, n_min: int = 2,
               workspace: Optional[torch.Tensor] = None) -> FitResult:
    """The k-dimensional Gaussian copula of eq. (7) by pseudo-likelihood per
    subset from doubled ranks R (k x n int32, as made by rank_margins;
    2 <= k <= 8), combined per group and parameter by eq. (15). The result is
    parameter-major: entry q K + m is correlation q (order (0,1), (0,2), ...,
    (k-2,k-1)) of subset m; combined entry q G + g."""
    R = _dev(R, "R")
    if R.dim() != 2:
        raise ValueError("R must be k x n")
    k, n = int(R.shape[0]), int(R.shape[1])
    p = k * (k - 1) // 2
    offsets = _i64(offsets)
    K = offsets.shape[0] - 1
    gofs = _i64(group_offsets if group_offsets is not None else [0, K])
    G = gofs.shape[0] - 1
    o = _options(n_min=n_min)
    nbytes = int(lib().cpc_gaussk_workspace_bytes(n, k, K, G))
    ws = _workspace(max(nbytes, 1), R.device, workspace)
    out = FitResult(torch.empty((max(p, 1) * K, 6), dtype=torch.float64, device=R.device),
                    torch.empty((max(p, 1) * G, 5), dtype=torch.float64, device=R.device))
    check(lib().cpc_gaussk_fit(_handle(R.device), R.data_ptr(), n, k, offsets.ctypes.data, K, gofs.ctypes.data, G,
                               ctypes.byref(o), ws.data_ptr(), ws.numel() * ws.element_size(), out.raw.data_ptr(),
                               out.raw_comb.data_ptr(), _stream(R.device)))
    return out
