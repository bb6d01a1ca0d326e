"""Plain FP64 CPU oracle for Tucker-ALS (HOOI) -- TEST INFRASTRUCTURE, NOT PRODUCT CODE.

Only the tests, the smoke check and the benchmark's CPU-baseline leg may import this
module.  It shares no code with the HIP library: it is written directly from the
paper's Sec. III-B with numpy in float64, one step at a time, so that a reader can
check it against the equations by eye.

Paper passages followed (Sharma & Grover, arXiv 2104.04726):

* Tucker model, eq. (1)-(2): X ~ Q x_1 S(1) x_2 S(2) ... x_N S(N), core Q of size
  R_1 x ... x R_N, factors S(n) of size s_n x R_n with orthonormal columns.
* T-HOSVD initialisation, Sec. III-B.1, eq. (3)-(7): the kept factor of mode r is the
  block of leading k_r left singular vectors of the mode-r unfolding of the data tensor
  (eq. (6)), and the truncated core is the data projected on those bases (eq. (7)).
  The interlaced HOSVD that the same section offers as a cheaper start is read as the
  sequentially truncated HOSVD: each mode's factor from the tensor already projected on the
  earlier modes' factors.
* HOOI sweep, Sec. III-B, eq. (8): for each mode n, Y(n) = X x_{m != n} S(m)^T, then S(n)
  takes the R_n leading left singular vectors of Y(n)_(n), obtained as the leading
  eigenvectors of the Gram matrix Y(n)_(n) Y(n)_(n)^T (the text right after eq. (8)).

Readings where the paper is silent or garbled:

* eq. (4) says the HOSVD factor is "the SVD of the unfolding of Q"; it is read as the left
  singular vectors of the unfolding of the *data* tensor, which is what eq. (6)-(7) use.
* The truncated core of eq. (7) is typed s_1 x ... x s_N; it is k_1 x ... x k_N.
* Sweep order is ascending 1..N and each update uses the newest factors (Gauss-Seidel).
* When R_n = s_n the factor is any orthonormal basis of R^{s_n}; the update is skipped.
* The core is formed once per sweep, after the last mode.
* fit = 1 - ||X - Xhat||_F / ||X||_F, evaluated as 1 - sqrt(max(||X||^2 - ||G||^2, 0)) / ||X||
  (valid because the factors are orthonormal); ||X|| = 0 gives fit = 1.
* Stopping: after max_iters sweeps, or earlier when |fit_k - fit_{k-1}| < tol (tol > 0),
  with fit_0 the T-HOSVD fit.

Conventions (Kolda-Bader): (X x_n M)[..., j, ...] = sum_i X[..., i, ...] M[j, i];
the mode-n unfolding is moveaxis(X, n, 0).reshape(s_n, -1) (its column order does not
affect Grams or left singular vectors).  Modes are 0-based in code.

Pins: every function here is checked in tests/test_oracle_pins.py against closed forms,
library routines (full SVD) or invariants that do not reuse this code.
"""

from __future__ import annotations

from dataclasses import dataclass, field
import math

import numpy as np


# --------------------------------------------------------------------------
# Validation (the same rules the library applies)
# --------------------------------------------------------------------------

def validate(dims, ranks, max_iters=0, tol=0.0):
    """Raise ValueError unless the problem is well posed.

    R_n must lie in [1, s_n], and R_n <= prod_{m != n} R_m: otherwise the mode-n Gram
    of Y(n) has rank < R_n and its leading R_n-dimensional subspace is not determined.
    """
    dims = [int(d) for d in dims]
    ranks = [int(r) for r in ranks]
    if not 2 <= len(dims) <= 8 or len(ranks) != len(dims):
        raise ValueError("order must be 2..8 and len(ranks) == len(dims)")
    for s, r in zip(dims, ranks):
        if s < 1 or r < 1 or r > s:
            raise ValueError("need 1 <= R_n <= s_n")
    total = math.prod(ranks)
    for r in ranks:
        if r * r > total:
            raise ValueError("need R_n <= prod of the other ranks")
    if max_iters < 0 or not (tol >= 0.0):
        raise ValueError("need max_iters >= 0 and tol >= 0")


# --------------------------------------------------------------------------
# Multilinear algebra (definitions written out)
# --------------------------------------------------------------------------

def unfold(x: np.ndarray, n: int) -> np.ndarray:
    """Mode-n unfolding X_(n): s_n rows, one column per index of the other modes."""
    return np.moveaxis(x, n, 0).reshape(x.shape[n], -1)


def ttm(x: np.ndarray, m: np.ndarray, n: int) -> np.ndarray:
    """Mode-n product X x_n M with M of shape (J, s_n): sum over the mode-n index."""
    if m.shape[1] != x.shape[n]:
        raise ValueError("inner dimensions differ")
    y = np.tensordot(m, x, axes=([1], [n]))       # new axis first
    return np.moveaxis(y, 0, n)


def project_all_but(x: np.ndarray, factors, skip: int) -> np.ndarray:
    """Y(n) = X x_{m != n} S(m)^T (eq. (8)), contracting modes in ascending order."""
    y = x
    for m, u in enumerate(factors):
        if m != skip:
            y = ttm(y, u.T, m)
    return y


def project_all(x: np.ndarray, factors) -> np.ndarray:
    """Core: X x_1 S(1)^T ... x_N S(N)^T (eq. (7) with the truncated bases)."""
    y = x
    for m, u in enumerate(factors):
        y = ttm(y, u.T, m)
    return y


def reconstruct(core: np.ndarray, factors) -> np.ndarray:
    """Xhat = Q x_1 S(1) ... x_N S(N) (eq. (1))."""
    y = core
    for m, u in enumerate(factors):
        y = ttm(y, u, m)
    return y


def gram(y: np.ndarray, n: int) -> np.ndarray:
    """Y_(n) Y_(n)^T, the mode-n Gram matrix."""
    yn = unfold(y, n)
    return yn @ yn.T


def leading_eigvecs(s: np.ndarray, r: int):
    """The r leading eigenvectors of a symmetric matrix (LAPACK eigh), largest first.

    Returns (U, lam) with lam all eigenvalues in descending order.
    """
    lam, v = np.linalg.eigh(s)
    order = np.argsort(lam)[::-1]
    lam = lam[order]
    v = v[:, order]
    return np.ascontiguousarray(v[:, :r]), lam


def fit_from_norms(nx2: float, ng2: float) -> float:
    """fit = 1 - ||X - Xhat|| / ||X||, using ||X - Xhat||^2 = ||X||^2 - ||G||^2."""
    if nx2 <= 0.0:
        return 1.0
    return 1.0 - math.sqrt(max(nx2 - ng2, 0.0)) / math.sqrt(nx2)


def identity_factors(dims, ranks):
    return [np.eye(s, r) for s, r in zip(dims, ranks)]


# --------------------------------------------------------------------------
# T-HOSVD and HOOI
# --------------------------------------------------------------------------

def thosvd_factors(x: np.ndarray, ranks):
    """Sec. III-B.1: S(n) = leading R_n left singular vectors of X_(n), via its Gram.

    Returns (factors, spectra) where spectra[n] are the Gram eigenvalues (descending).
    """
    factors, spectra = [], []
    for n, r in enumerate(ranks):
        u, lam = leading_eigvecs(gram(x, n), r)
        factors.append(u)
        spectra.append(lam)
    return factors, spectra


def st_hosvd_factors(x: np.ndarray, ranks):
    """Sequentially truncated ("interlaced") HOSVD, the cheaper start the paper names after eq. (7).

    Modes are taken in ascending order.  S(n) = leading R_n left singular vectors of the mode-n
    unfolding of the tensor already projected on the earlier factors,
    Y(n-1) = X x_1 S(1)^T ... x_{n-1} S(n-1)^T (via its Gram), and Y(n) = Y(n-1) x_n S(n)^T; the
    core of the start is Y(N).  Returns (factors, spectra, core) with spectra[n] the eigenvalues of
    the Gram of Y(n-1)_(n), descending.  R_n = s_n keeps the identity basis: it spans all of R^{s_n}.
    """
    y = x
    factors, spectra = [], []
    for n, r in enumerate(ranks):
        s_n = gram(y, n)
        if r == x.shape[n]:
            u, lam = np.eye(r), np.linalg.eigvalsh(s_n)[::-1]
        else:
            u, lam = leading_eigvecs(s_n, r)
        factors.append(u)
        spectra.append(lam)
        y = ttm(y, u.T, n)
    return factors, spectra, y


def hooi_update(x: np.ndarray, factors, n: int, rank: int):
    """One factor update of eq. (8): Y = X x_{m != n} S(m)^T, S(n) <- top-R_n eigvecs of Y_(n)Y_(n)^T.

    Returns (new factor, Gram eigenvalues descending, Y).  R_n = s_n keeps the old factor.
    """
    y = project_all_but(x, factors, n)
    if rank == x.shape[n]:
        lam = np.linalg.eigvalsh(gram(y, n))[::-1]
        return factors[n], lam, y
    u, lam = leading_eigvecs(gram(y, n), rank)
    return u, lam, y


@dataclass
class HooiResult:
    core: np.ndarray
    factors: list
    fits: list                      # fits[0] = T-HOSVD fit, fits[k] after sweep k
    sweeps: int
    norm_x2: float
    spectra: list = field(default_factory=list)   # last Gram eigenvalues per mode

    def gap_factor(self, n: int, rank: int) -> float:
        """g_n = lam_1 / (lam_R - lam_{R+1}) of the last mode-n Gram (inf for a tie)."""
        lam = self.spectra[n]
        if rank >= len(lam):
            return 0.0
        gap = lam[rank - 1] - lam[rank]
        return float(lam[0] / gap) if gap > 0 else math.inf


def hooi(x: np.ndarray, ranks, max_iters: int = 10, tol: float = 0.0, init=None,
         start: str = "thosvd") -> HooiResult:
    """Tucker-ALS by HOOI, FP64.

    init: optional list of orthonormal factors replacing the start (resume).
    start: "thosvd" (every factor from the unprojected X, Sec. III-B.1) or "sthosvd" (the
    sequentially truncated / interlaced HOSVD, st_hosvd_factors).
    """
    x = np.asarray(x, dtype=np.float64)
    ranks = [int(r) for r in ranks]
    validate(x.shape, ranks, max_iters, tol)
    if start not in ("thosvd", "sthosvd"):
        raise ValueError("start must be 'thosvd' or 'sthosvd'")
    nx2 = float(np.sum(x * x))
    if nx2 == 0.0:
        factors = identity_factors(x.shape, ranks)
        return HooiResult(np.zeros(ranks), factors, [1.0], 0, 0.0,
                          [np.zeros(s) for s in x.shape])
    if init is None and start == "sthosvd":
        factors, spectra, _ = st_hosvd_factors(x, ranks)
    elif init is None:
        factors, spectra = thosvd_factors(x, ranks)
    else:
        factors = [np.array(u, dtype=np.float64, copy=True) for u in init]
        spectra = [np.linalg.eigvalsh(gram(x, n))[::-1] for n in range(x.ndim)]
    core = project_all(x, factors)
    fits = [fit_from_norms(nx2, float(np.sum(core * core)))]
    sweeps = 0
    for _ in range(max_iters):
        y = None
        for n, r in enumerate(ranks):
            u, lam, y = hooi_update(x, factors, n, r)
            factors[n] = u
            spectra[n] = lam
        # core after the last mode: G = Y(N) x_N S(N)^T
        core = ttm(y, factors[-1].T, x.ndim - 1)
        fits.append(fit_from_norms(nx2, float(np.sum(core * core))))
        sweeps += 1
        if tol > 0.0 and abs(fits[-1] - fits[-2]) < tol:
            break
    return HooiResult(core, factors, fits, sweeps, nx2, spectra)


def sign_fix(core: np.ndarray, factors):
    """Make each factor column's largest-magnitude entry positive, flipping the core to match.

    Xhat is unchanged; used only to print deterministic factors.
    """
    core = core.copy()
    out = []
    for n, u in enumerate(factors):
        idx = np.argmax(np.abs(u), axis=0)
        sg = np.sign(u[idx, np.arange(u.shape[1])])
        sg[sg == 0] = 1.0
        out.append(u * sg[None, :])
        shape = [1] * core.ndim
        shape[n] = -1
        core = core * sg.reshape(shape)
    return core, out
