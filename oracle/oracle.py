"""ctypes wrapper of the plain FP64 CPU oracle (``cpc_oracle.c``).

TEST INFRASTRUCTURE. Only the test suite, ``__graft_entry__.smoke()`` and the
CPU-baseline leg of ``bench.py`` may import this module. It never touches the
GPU library and the GPU library never touches it.

The oracle follows arXiv:1609.05530: ranks by eq. (12) with N read as the
subset size, the pseudo log-likelihood of eq. (13) for the copulas of eq. (8),
(10) and (11) (densities by eq. (5)), its numerical maximisation and the
Genest-Ghoudi-Rivest asymptotic variance (Sec. 2.3), the row partition of
eq. (14) and the inverse-variance combination of eq. (15)/(16).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(_HERE, "cpc_oracle.c")
LIB = os.path.join(_HERE, "liboracle.so")

FAMILIES = {"gaussian": 0, "frank": 1, "gumbel": 2}
TIES = {"average": 0, "first": 1}
VARS = {"ggr": 0, "invinfo": 1}

STATUS_NAMES = {
    0: "OK",
    1: "BOUNDARY_NATURAL",
    2: "BOUNDARY_BOX",
    3: "DEGENERATE",
    4: "NONFINITE",
    5: "NOCONV",
    6: "BADVAR",
}

SUBSET_DTYPE = np.dtype(
    [("theta", "f8"), ("var", "f8"), ("loglik", "f8"), ("score", "f8"), ("n", "i8"),
     ("iters", "i4"), ("status", "i4")], align=True)
COMBINED_DTYPE = np.dtype(
    [("theta", "f8"), ("var_combined", "f8"), ("n_used", "i8"), ("n_excluded", "i8"),
     ("status", "i4"), ("pad", "i4")], align=True)


class _Options(ctypes.Structure):
    _fields_ = [("ties", ctypes.c_int32), ("var", ctypes.c_int32), ("max_iter", ctypes.c_int32),
                ("pad", ctypes.c_int32), ("tol", ctypes.c_double), ("n_min", ctypes.c_int64)]


def build() -> str:
    """Compile the oracle with gcc (IEEE double, no fast-math, no FMA contraction)."""
    cmd = ["gcc", "-O2", "-std=c11", "-ffp-contract=off", "-fopenmp", "-fPIC", "-shared",
           "-o", LIB + ".tmp", SRC, "-lm"]
    subprocess.check_call(cmd, cwd=_HERE)
    os.replace(LIB + ".tmp", LIB)
    return LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
            build()
        L = ctypes.CDLL(LIB)
        d = ctypes.c_double
        i32 = ctypes.c_int32
        i64 = ctypes.c_int64
        p = ctypes.c_void_p
        L.or_qnorm.restype = d
        L.or_qnorm.argtypes = [d, d]
        L.or_tau.restype = d
        L.or_tau.argtypes = [i32, d]
        L.or_rho_s.restype = d
        L.or_rho_s.argtypes = [i32, d]
        L.or_debye.restype = d
        L.or_debye.argtypes = [i32, d]
        L.or_ranks.restype = None
        L.or_ranks.argtypes = [p, i64, i32, p]
        L.or_logc_derivs.restype = None
        L.or_logc_derivs.argtypes = [i32, d, p, p, p, p, i64, p]
        L.or_ggr.restype = d
        L.or_ggr.argtypes = [p, p, i64, i32, d, i32, p]
        L.or_combine.restype = None
        L.or_combine.argtypes = [p, p, i64, p]
        L.or_fit.restype = None
        L.or_fit.argtypes = [p, p, p, i64, p, i64, p, ctypes.POINTER(_Options), i32, p, p]
        L.or_num_threads.restype = i32
        L.or_num_threads.argtypes = [i32]
        L.or_philox4x32_10.restype = None
        L.or_philox4x32_10.argtypes = [p, p, p]
        L.or_sample.restype = None
        L.or_sample.argtypes = [i32, d, ctypes.c_uint64, i64, i64, p, p]
        L.or_density_distance.restype = None
        L.or_density_distance.argtypes = [i32, d, d, d, i32, i32, p]
        L.or_spearman.restype = d
        L.or_spearman.argtypes = [p, p, i64]
        L.or_spearman_theta.restype = d
        L.or_spearman_theta.argtypes = [i32, d, p]
        L.or_spearman_var.restype = d
        L.or_spearman_var.argtypes = [p, p, i64, i32, d, p]
        L.or_spearman_fit_ranks.restype = None
        L.or_spearman_fit_ranks.argtypes = [p, p, i64, i32, i64, p]
        L.or_kendall_rows.restype = None
        L.or_kendall_rows.argtypes = [p, p, i64, p]
        L.or_kendall.restype = d
        L.or_kendall.argtypes = [p, p, i64]
        L.or_tau_slope.restype = d
        L.or_tau_slope.argtypes = [i32, d]
        L.or_kendall_theta.restype = d
        L.or_kendall_theta.argtypes = [i32, d, p]
        L.or_kendall_var.restype = d
        L.or_kendall_var.argtypes = [p, p, i64, i32, d, p, p]
        L.or_kendall_fit_ranks.restype = None
        L.or_kendall_fit_ranks.argtypes = [p, p, i64, i32, i64, p]
        _lib = L
    return _lib


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def _fam(f) -> int:
    return FAMILIES[f] if isinstance(f, str) else int(f)


def qnorm(p, omp=None) -> np.ndarray:
    p = np.atleast_1d(np.asarray(p, dtype=np.float64))
    omp = 1.0 - p if omp is None else np.atleast_1d(np.asarray(omp, dtype=np.float64))
    L = lib()
    return np.array([L.or_qnorm(float(a), float(b)) for a, b in zip(p, omp)])


def tau(family, theta: float) -> float:
    return lib().or_tau(_fam(family), float(theta))


def rho_s(family, theta: float) -> float:
    return lib().or_rho_s(_fam(family), float(theta))


def debye(k: int, x: float) -> float:
    return lib().or_debye(int(k), float(x))


def ranks(x, ties: str = "average") -> np.ndarray:
    """Doubled ranks R = 2 * rank of eq. (12) (average ties stay integer)."""
    x = np.ascontiguousarray(x, dtype=np.float64)
    R = np.empty(x.shape[0], dtype=np.int64)
    lib().or_ranks(_ptr(x), x.shape[0], TIES[ties], _ptr(R))
    return R


def pobs_from_ranks(R: np.ndarray, n: int):
    """u = R / (2(n+1)) and 1 - u = (2(n+1) - R) / (2(n+1)), both exact rationals."""
    den = 2.0 * (n + 1.0)
    R = np.asarray(R, dtype=np.float64)
    return R / den, (den - R) / den


def logc_derivs(family, theta: float, u, omu, v, omv) -> np.ndarray:
    """Per row: l, l_theta, l_theta_theta, l_theta_u, l_theta_v (shape (n, 5))."""
    arrs = [np.ascontiguousarray(a, dtype=np.float64) for a in (u, omu, v, omv)]
    n = arrs[0].shape[0]
    out = np.empty((n, 5), dtype=np.float64)
    lib().or_logc_derivs(_fam(family), float(theta), *[_ptr(a) for a in arrs], n, _ptr(out))
    return out


def ggr(R1, R2, family, theta: float, var: str = "ggr"):
    """GGR plug-in variance at theta; also returns per-row (s, W1, W2, psi)."""
    R1 = np.ascontiguousarray(R1, dtype=np.int64)
    R2 = np.ascontiguousarray(R2, dtype=np.int64)
    n = R1.shape[0]
    terms = np.empty((n, 4), dtype=np.float64)
    v = lib().or_ggr(_ptr(R1), _ptr(R2), n, _fam(family), float(theta), VARS[var], _ptr(terms))
    return v, terms


def options(ties="average", var="ggr", max_iter=100, tol=1e-13, n_min=2) -> _Options:
    return _Options(TIES[ties], VARS[var], int(max_iter), 0, float(tol), int(n_min))


def fit(x, y, offsets, family, group_offsets=None, *, ties="average", var="ggr", max_iter=100,
        tol=1e-13, n_min=2, nthreads=0):
    """Fit every subset [offsets[m], offsets[m+1]) and combine per group.

    ``family`` is one family (all groups) or a sequence with one per group.
    Returns (subsets, combined) as numpy structured arrays.
    """
    x = np.ascontiguousarray(x, dtype=np.float64)
    y = np.ascontiguousarray(y, dtype=np.float64)
    offsets = np.ascontiguousarray(offsets, dtype=np.int64)
    K = offsets.shape[0] - 1
    if group_offsets is None:
        group_offsets = np.array([0, K], dtype=np.int64)
    group_offsets = np.ascontiguousarray(group_offsets, dtype=np.int64)
    G = group_offsets.shape[0] - 1
    if isinstance(family, (str, int, np.integer)):
        fams = np.full(G, _fam(family), dtype=np.int32)
    else:
        fams = np.ascontiguousarray([_fam(f) for f in family], dtype=np.int32)
    sub = np.zeros(K, dtype=SUBSET_DTYPE)
    comb = np.zeros(G, dtype=COMBINED_DTYPE)
    opt = options(ties, var, max_iter, tol, n_min)
    lib().or_fit(_ptr(x), _ptr(y), _ptr(offsets), K, _ptr(group_offsets), G, _ptr(fams),
                 ctypes.byref(opt), int(nthreads), _ptr(sub), _ptr(comb))
    return sub, comb


def combine(sub: np.ndarray, group_offsets) -> np.ndarray:
    sub = np.ascontiguousarray(sub, dtype=SUBSET_DTYPE)
    group_offsets = np.ascontiguousarray(group_offsets, dtype=np.int64)
    G = group_offsets.shape[0] - 1
    comb = np.zeros(G, dtype=COMBINED_DTYPE)
    lib().or_combine(_ptr(sub), _ptr(group_offsets), G, _ptr(comb))
    return comb


def num_threads(requested: int = 0) -> int:
    return lib().or_num_threads(int(requested))


# --------------------------------------------------------------------------
# Simulation inputs and the evaluation metrics of Sec. 2.5-2.6.

def philox4x32_10(ctr, key) -> np.ndarray:
    """Philox4x32-10 block of a 4-word counter and a 2-word key."""
    c = np.ascontiguousarray(ctr, dtype=np.uint32)
    k = np.ascontiguousarray(key, dtype=np.uint32)
    out = np.empty(4, dtype=np.uint32)
    lib().or_philox4x32_10(_ptr(c), _ptr(k), _ptr(out))
    return out


def sample(family, theta: float, seed: int, row0: int, n: int):
    """Rows row0 .. row0+n-1 of the seeded stream of pairs with N(0,1)
    margins and the family's copula at theta (the GPU sampler's definition)."""
    x = np.empty(n, dtype=np.float64)
    y = np.empty(n, dtype=np.float64)
    lib().or_sample(_fam(family), float(theta), ctypes.c_uint64(int(seed)), int(row0), int(n), _ptr(x), _ptr(y))
    return x, y


def density_distance(family, theta_a: float, theta_b: float, box: float = 20.0, panels: int = 64,
                     nodes: int = 16) -> np.ndarray:
    """[int |c_a - c_b|, int c_a, int (c_a - c_b)^2, int c_a^2] over the unit
    square (eq. 19 = [0]/[1], eq. 20 = sqrt([2]/[3])), in normal-score
    coordinates over |s|, |t| <= box."""
    out = np.empty(4, dtype=np.float64)
    lib().or_density_distance(_fam(family), float(theta_a), float(theta_b), float(box), int(panels), int(nodes),
                              _ptr(out))
    return out


def replicate_summary(comb_theta, comb_status, full_theta, full_status) -> np.ndarray:
    """Sec. 2.6 over the replicates whose combined (eq. 16) and full-data
    estimates both have status 0: [eq. (17), eq. (18), bias, MSE, count]."""
    ct = np.asarray(comb_theta, dtype=np.float64)
    ft = np.asarray(full_theta, dtype=np.float64)
    use = (np.asarray(comb_status) == 0) & (np.asarray(full_status) == 0)
    s = int(use.sum())
    mc = float(np.sum(ct[use]) / s)
    mf = float(np.sum(ft[use]) / s)
    mse = float(np.sum((ct[use] - ft[use]) ** 2) / s)
    return np.array([mc, mf, mc - mf, mse, float(s)])


# --------------------------------------------------------------------------
# The inversion of Spearman's rho as an estimator (Sec. 2.3).

def spearman(R1, R2) -> float:
    """rho_S hat from doubled ranks."""
    R1 = np.ascontiguousarray(R1, dtype=np.int64)
    R2 = np.ascontiguousarray(R2, dtype=np.int64)
    return lib().or_spearman(_ptr(R1), _ptr(R2), R1.shape[0])


def spearman_theta(family, r: float):
    """theta with rho_S(theta) = r, and the status (0, 1 natural boundary, 2 box edge)."""
    st = ctypes.c_int32()
    th = lib().or_spearman_theta(_fam(family), float(r), ctypes.byref(st))
    return th, st.value


def spearman_var(R1, R2, family, theta: float):
    """(variance of the estimate, var(psi)) at theta."""
    R1 = np.ascontiguousarray(R1, dtype=np.int64)
    R2 = np.ascontiguousarray(R2, dtype=np.int64)
    nu = ctypes.c_double()
    v = lib().or_spearman_var(_ptr(R1), _ptr(R2), R1.shape[0], _fam(family), float(theta), ctypes.byref(nu))
    return v, nu.value


def spearman_fit_ranks(R1, R2, offsets, family, group_offsets=None, n_min=2):
    """Per subset from doubled ranks, and the combination of eq. (15) per group."""
    R1 = np.ascontiguousarray(R1, dtype=np.int64)
    R2 = np.ascontiguousarray(R2, dtype=np.int64)
    offsets = np.ascontiguousarray(offsets, dtype=np.int64)
    K = offsets.shape[0] - 1
    if group_offsets is None:
        group_offsets = np.array([0, K], dtype=np.int64)
    group_offsets = np.ascontiguousarray(group_offsets, dtype=np.int64)
    G = group_offsets.shape[0] - 1
    fams = [family] * G if isinstance(family, (str, int, np.integer)) else list(family)
    sub = np.zeros(K, dtype=SUBSET_DTYPE)
    L = lib()
    for g in range(G):
        for m in range(group_offsets[g], group_offsets[g + 1]):
            a, b = offsets[m], offsets[m + 1]
            one = np.zeros(1, dtype=SUBSET_DTYPE)
            L.or_spearman_fit_ranks(_ptr(R1[a:b]), _ptr(R2[a:b]), b - a, _fam(fams[g]), int(n_min), _ptr(one))
            sub[m] = one[0]
    return sub, combine(sub, group_offsets)


# --------------------------------------------------------------------------
# The inversion of Kendall's tau as an estimator (Sec. 2.3).

def kendall_rows(R1, R2) -> np.ndarray:
    """S_i = sum over l != i of sign(r1_i - r1_l) sign(r2_i - r2_l)."""
    R1 = np.ascontiguousarray(R1, dtype=np.int64)
    R2 = np.ascontiguousarray(R2, dtype=np.int64)
    S = np.zeros(R1.shape[0], dtype=np.int64)
    lib().or_kendall_rows(_ptr(R1), _ptr(R2), R1.shape[0], _ptr(S))
    return S


def kendall(R1, R2) -> float:
    """tau hat from doubled ranks."""
    R1 = np.ascontiguousarray(R1, dtype=np.int64)
    R2 = np.ascontiguousarray(R2, dtype=np.int64)
    return lib().or_kendall(_ptr(R1), _ptr(R2), R1.shape[0])


def tau_slope(family, theta: float) -> float:
    return lib().or_tau_slope(_fam(family), float(theta))


def kendall_theta(family, t: float):
    """theta with tau(theta) = t, and the status (0, 1 natural boundary, 2 box edge)."""
    st = ctypes.c_int32()
    th = lib().or_kendall_theta(_fam(family), float(t), ctypes.byref(st))
    return th, st.value


def kendall_var(R1, R2, family, theta: float):
    """(variance of the estimate, var(k1), tau hat) at theta."""
    R1 = np.ascontiguousarray(R1, dtype=np.int64)
    R2 = np.ascontiguousarray(R2, dtype=np.int64)
    zeta, t = ctypes.c_double(), ctypes.c_double()
    v = lib().or_kendall_var(_ptr(R1), _ptr(R2), R1.shape[0], _fam(family), float(theta), ctypes.byref(zeta),
                             ctypes.byref(t))
    return v, zeta.value, t.value


def kendall_fit_ranks(R1, R2, offsets, family, group_offsets=None, n_min=2):
    """Per subset from doubled ranks, and the combination of eq. (15) per group."""
    R1 = np.ascontiguousarray(R1, dtype=np.int64)
    R2 = np.ascontiguousarray(R2, dtype=np.int64)
    offsets = np.ascontiguousarray(offsets, dtype=np.int64)
    K = offsets.shape[0] - 1
    if group_offsets is None:
        group_offsets = np.array([0, K], dtype=np.int64)
    group_offsets = np.ascontiguousarray(group_offsets, dtype=np.int64)
    G = group_offsets.shape[0] - 1
    fams = [family] * G if isinstance(family, (str, int, np.integer)) else list(family)
    sub = np.zeros(K, dtype=SUBSET_DTYPE)
    L = lib()
    for g in range(G):
        for m in range(group_offsets[g], group_offsets[g + 1]):
            a, b = offsets[m], offsets[m + 1]
            one = np.zeros(1, dtype=SUBSET_DTYPE)
            L.or_kendall_fit_ranks(_ptr(R1[a:b]), _ptr(R2[a:b]), b - a, _fam(fams[g]), int(n_min), _ptr(one))
            sub[m] = one[0]
    return sub, combine(sub, group_offsets)
