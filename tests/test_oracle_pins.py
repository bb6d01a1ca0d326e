"""Pins of the FP64 oracle against facts that do not come from the oracle itself.

Each check uses an independent route: closed forms, numpy's full SVD of explicitly
built unfoldings, einsum reconstructions written here, or invariants of HOOI
(Sec. III-B of arXiv 2104.04726).  The last group plants mistakes in a copy of the
oracle and checks that the pins catch them.
"""

import itertools
import json
import math
import os

import numpy as np
import pytest

import oracle
from oracle import hooi_ref
from synth import make_exact_rank, make_tiny, make_stereo_stack, STACK_CONFIGS

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


# ---------------------------------------------------------------- independent helpers

def einsum_reconstruct(core, factors):
    """Xhat[i,j,...] = sum_r G[r...] prod_n U_n[i_n, r_n], written with one einsum."""
    letters_r = "abcdefgh"[: core.ndim]
    letters_i = "ijklmnop"[: core.ndim]
    spec = letters_r + "," + ",".join(i + r for i, r in zip(letters_i, letters_r)) + "->" + letters_i
    return np.einsum(spec, core, *factors, optimize=True)


def einsum_project(x, factors, skip=None):
    """X x_{m != skip} U_m^T with one einsum (the skipped mode keeps its index)."""
    nd = x.ndim
    li = "ijklmnop"[:nd]
    lr = "abcdefgh"[:nd]
    out = "".join(li[m] if m == skip else lr[m] for m in range(nd))
    ops = [x]
    spec = li
    for m in range(nd):
        if m == skip:
            continue
        spec += "," + li[m] + lr[m]
        ops.append(factors[m])
    return np.einsum(spec + "->" + out, *ops, optimize=True)


def loop_unfold(x, n):
    """Mode-n unfolding built by an explicit loop over all entries (tiny tensors only)."""
    shape = x.shape
    others = [m for m in range(x.ndim) if m != n]
    cols = list(itertools.product(*[range(shape[m]) for m in others]))
    out = np.zeros((shape[n], len(cols)))
    for c, idx in enumerate(cols):
        for i in range(shape[n]):
            full = [0] * x.ndim
            full[n] = i
            for m, v in zip(others, idx):
                full[m] = v
            out[i, c] = x[tuple(full)]
    return out


def svd_left(a, r):
    u, s, _ = np.linalg.svd(a, full_matrices=False)
    return u[:, :r], s


def sin_theta(a, b):
    d = a - b @ (b.T @ a)
    return float(np.linalg.norm(d, 2)) if d.size else 0.0


def rel_resid(x, core, factors):
    return float(np.linalg.norm(x - einsum_reconstruct(core, factors)) / np.linalg.norm(x))


def gapped_random(dims, ranks, seed, noise=1e-2):
    x, _, _ = make_exact_rank(dims, ranks, seed, noise)
    return x


# ---------------------------------------------------------------- golden closed forms

def test_golden_superdiagonal():
    g = json.load(open(os.path.join(GOLDEN, "superdiag_2x2x2.json")))
    x = np.zeros(g["dims"])
    for *idx, v in g["entries"]:
        x[tuple(idx)] = v
    res = oracle.hooi(x, g["ranks"], max_iters=3)
    assert abs(res.fits[0] - g["fit"]) < 1e-14
    assert abs(res.fits[-1] - g["fit"]) < 1e-14
    assert abs(abs(res.core.item()) - g["core_abs"]) < 1e-14


@pytest.mark.parametrize("case", [0, 1, 2])
def test_golden_orthogonally_decomposable(case):
    g = json.load(open(os.path.join(GOLDEN, "odeco_3x3x3.json")))
    a, b, c = (np.array(g[k]) for k in "abc")
    sig = g["sigma"]
    x = sum(s * np.einsum("i,j,k->ijk", a[r], b[r], c[r]) for r, s in enumerate(sig))
    cs = g["cases"][case]
    res = oracle.hooi(x, cs["ranks"], max_iters=2)
    # fit via the explicit residual (the norm formula loses half the digits near fit = 1)
    fit_explicit = 1.0 - rel_resid(x, res.core, res.factors)
    assert abs(fit_explicit - cs["fit"]) < 1e-12
    assert abs(res.fits[0] - cs["fit"]) < 1e-7
    got = sorted(np.abs(res.core).ravel())[::-1][: len(cs["core_abs_sorted"])]
    np.testing.assert_allclose(got, cs["core_abs_sorted"], atol=1e-12)


# ---------------------------------------------------------------- P1 exact multilinear rank

@pytest.mark.parametrize("seed", [0, 1])
def test_p1_exact_rank_recovery(seed):
    x, core, fac = make_exact_rank((12, 10, 4, 5), (3, 4, 2, 3), seed, 0.0)
    res = oracle.hooi(x, (3, 4, 2, 3), max_iters=3)
    assert rel_resid(x, res.core, res.factors) < 1e-12
    assert res.fits[-1] > 1.0 - 1e-7
    for u, t in zip(res.factors, fac):
        assert sin_theta(u, t) < 1e-10


# ---------------------------------------------------------------- P2 noisy tiny case

def test_p2_tiny_noise_perturbation():
    noise_rel = 1e-3
    x, core, fac = make_tiny(0, noise_rel)
    x0, _, _ = make_tiny(0, 0.0)
    res = oracle.hooi(x, (16, 12, 3, 4), max_iters=10)
    dims, ranks = x.shape, (16, 12, 3, 4)
    sig_e = noise_rel * math.sqrt(float(np.mean(x0 * x0)))
    for n in range(4):
        s_n = dims[n]
        others = math.prod(dims) // s_n
        # Wedin: sin theta <= ||E_(n)|| / (sigma_R(X0_(n)) - ||E_(n)||); Gaussian E: ||E_(n)|| ~ sig (sqrt s + sqrt others)
        e_norm = sig_e * (math.sqrt(s_n) + math.sqrt(others))
        smin = np.linalg.svd(loop_unfold(x0, n) if x0.size < 1000 else np.moveaxis(x0, n, 0).reshape(s_n, -1),
                             compute_uv=False)[ranks[n] - 1]
        bound = e_norm / (smin - e_norm)
        st = sin_theta(res.factors[n], fac[n])
        if ranks[n] == s_n:
            assert st < 1e-12
        else:
            assert st <= 10 * bound, (n, st, bound)
    # residual ~ the noise outside the fitted model: sigma * sqrt(#entries - #model parameters)
    dof = math.prod(ranks) + sum(r * (s - r) for s, r in zip(dims, ranks))
    rho_expected = sig_e * math.sqrt(math.prod(dims) - dof) / np.linalg.norm(x)
    rho = 1.0 - res.fits[-1]
    assert abs(rho - rho_expected) < 0.05 * rho_expected, (rho, rho_expected)


# ---------------------------------------------------------------- P3 Pythagorean identity

def test_p3_pythagorean_every_sweep():
    x = gapped_random((9, 8, 7, 6), (4, 3, 3, 2), 5, noise=0.3)
    nx2 = float(np.sum(x * x))
    for k in range(0, 4):
        res = oracle.hooi(x, (4, 3, 3, 2), max_iters=k)
        xh = einsum_reconstruct(res.core, res.factors)
        lhs = nx2 - float(np.sum(res.core ** 2)) - float(np.sum((x - xh) ** 2))
        assert abs(lhs) <= 1e-12 * nx2


# ---------------------------------------------------------------- P4 monotone fit

@pytest.mark.parametrize("which", ["random", "stack"])
def test_p4_monotone_fit(which):
    if which == "random":
        x = gapped_random((10, 9, 8, 7), (4, 4, 3, 3), 3, noise=1.0)
        ranks = (4, 4, 3, 3)
    else:
        c = STACK_CONFIGS["stack_mini"]
        x = make_stereo_stack(90, 160, 3, "ycbcr", seed=4).astype(np.float64)
        ranks = (24, 32, 3, 4)
    res = oracle.hooi(x, ranks, max_iters=8)
    for k in range(1, len(res.fits)):
        assert res.fits[k] >= res.fits[k - 1] - 1e-13, (k, res.fits)


# ---------------------------------------------------------------- P5 brute-force SVD

def test_p5_init_and_updates_match_full_svd():
    x = gapped_random((6, 5, 4, 3), (3, 2, 2, 2), 7, noise=0.05)
    ranks = (3, 2, 2, 2)
    facs, _ = oracle.thosvd_factors(x, ranks)
    for n in range(4):
        u, s = svd_left(loop_unfold(x, n), ranks[n])
        assert s[ranks[n] - 1] - s[ranks[n]] > 1e-3
        assert sin_theta(facs[n], u) < 1e-12
    # each HOOI update against the SVD of an explicitly built Y_(n)
    cur = [f.copy() for f in facs]
    for n in range(4):
        new, _, _ = oracle.hooi_update(x, cur, n, ranks[n])
        y = einsum_project(x, cur, skip=n)
        u, s = svd_left(loop_unfold(y, n), ranks[n])
        if ranks[n] < x.shape[n]:
            assert sin_theta(new, u) < 1e-12
        cur[n] = new


# ---------------------------------------------------------------- P6 Eckart-Young (order 2)

def test_p6_eckart_young():
    rng = np.random.default_rng(9)
    x = rng.standard_normal((30, 20)) @ np.diag(np.linspace(3, 0.1, 20)) @ rng.standard_normal((20, 20))
    r = 5
    s = np.linalg.svd(x, compute_uv=False)
    expected = 1.0 - math.sqrt(float(np.sum(s[r:] ** 2))) / math.sqrt(float(np.sum(s ** 2)))
    res = oracle.hooi(x, (r, r), max_iters=3)
    assert abs(res.fits[0] - expected) < 1e-13
    assert abs(res.fits[1] - res.fits[0]) < 1e-13
    assert abs(res.fits[-1] - expected) < 1e-13


# ---------------------------------------------------------------- P7 full rank

def test_p7_full_rank_identity():
    x = gapped_random((5, 4, 3, 2), (2, 2, 2, 2), 1, noise=1.0)
    res = oracle.hooi(x, x.shape, max_iters=2)
    assert rel_resid(x, res.core, res.factors) < 1e-13
    assert res.fits[-1] > 1.0 - 1e-7


# ---------------------------------------------------------------- P8 rank one

def test_p8_rank_one_closed_form():
    rng = np.random.default_rng(2)
    vs = [rng.standard_normal(s) for s in (7, 6, 5, 4)]
    x = np.einsum("i,j,k,l->ijkl", *vs)
    res = oracle.hooi(x, (1, 1, 1, 1), max_iters=2)
    assert abs(abs(res.core.item()) - np.linalg.norm(x)) < 1e-13 * np.linalg.norm(x)
    for u, v in zip(res.factors, vs):
        assert sin_theta(u, (v / np.linalg.norm(v))[:, None]) < 1e-12


# ---------------------------------------------------------------- P9 truncation bounds

@pytest.mark.parametrize("k", [0, 1, 3])
def test_p9_truncation_bounds(k):
    x = make_stereo_stack(48, 64, 3, "ipt", seed=6).astype(np.float64)
    ranks = (12, 16, 3, 4)
    taus = []
    for n, r in enumerate(ranks):
        s = np.linalg.svd(np.moveaxis(x, n, 0).reshape(x.shape[n], -1), compute_uv=False)
        taus.append(float(np.sum(s[r:] ** 2)))
    res = oracle.hooi(x, ranks, max_iters=k)
    err2 = float(np.sum((x - einsum_reconstruct(res.core, res.factors)) ** 2))
    assert max(taus) <= err2 * (1 + 1e-10)
    assert err2 <= sum(taus) * (1 + 1e-10)


# ---------------------------------------------------------------- P10 stationarity

def test_p10_stationarity_after_convergence():
    x = gapped_random((10, 9, 8, 6), (3, 3, 2, 2), 11, noise=0.05)
    ranks = (3, 3, 2, 2)
    res = oracle.hooi(x, ranks, max_iters=60)
    for n in range(4):
        y = einsum_project(x, res.factors, skip=n)
        s = np.moveaxis(y, n, 0).reshape(x.shape[n], -1)
        s = s @ s.T
        u = res.factors[n]
        r = s @ u - u @ (u.T @ s @ u)
        assert np.linalg.norm(r) <= 1e-9 * np.linalg.norm(s)


# ---------------------------------------------------------------- P11 equivariances

def test_p11_equivariances():
    x = gapped_random((8, 7, 6, 5), (3, 3, 2, 2), 4, noise=0.05)
    ranks = (3, 3, 2, 2)
    base = oracle.hooi(x, ranks, max_iters=4)
    # mode permutation
    perm = (2, 0, 3, 1)
    pr = oracle.hooi(np.transpose(x, perm), [ranks[p] for p in perm], max_iters=4)
    assert abs(pr.fits[-1] - base.fits[-1]) < 1e-12
    # orthogonal change of basis in mode 1: U_1 -> Q U_1, same fit
    q, _ = np.linalg.qr(np.random.default_rng(0).standard_normal((7, 7)))
    xq = np.einsum("ijkl,aj->iakl", x, q)
    qr = oracle.hooi(xq, ranks, max_iters=4)
    assert abs(qr.fits[-1] - base.fits[-1]) < 1e-12
    assert sin_theta(qr.factors[1], q @ base.factors[1]) < 1e-10
    # scaling: same factors and fit, core scales
    sc = oracle.hooi(3.5 * x, ranks, max_iters=4)
    assert abs(sc.fits[-1] - base.fits[-1]) < 1e-12
    assert abs(np.linalg.norm(sc.core) - 3.5 * np.linalg.norm(base.core)) < 1e-12 * np.linalg.norm(sc.core)


# ---------------------------------------------------------------- P12 resume

def test_p12_resume_bitwise():
    x = gapped_random((9, 8, 5, 4), (3, 3, 2, 2), 8, noise=0.2)
    ranks = (3, 3, 2, 2)
    full = oracle.hooi(x, ranks, max_iters=5)
    part = oracle.hooi(x, ranks, max_iters=2)
    rest = oracle.hooi(x, ranks, max_iters=3, init=part.factors)
    for a, b in zip(full.factors, rest.factors):
        assert np.array_equal(a, b)
    assert np.array_equal(full.core, rest.core)
    assert full.fits[-1] == rest.fits[-1]


# ---------------------------------------------------------------- stopping rule and edge cases

def test_tol_stops_early_and_zero_tensor():
    x = gapped_random((8, 7, 6, 5), (3, 3, 2, 2), 4, noise=0.05)
    res = oracle.hooi(x, (3, 3, 2, 2), max_iters=50, tol=1e-9)
    assert res.sweeps < 50
    assert abs(res.fits[-1] - res.fits[-2]) < 1e-9
    z = oracle.hooi(np.zeros((4, 3, 2)), (2, 2, 1), max_iters=3)
    assert z.fits == [1.0] and not np.any(z.core)
    for u, s in zip(z.factors, (4, 3, 2)):
        assert np.array_equal(u, np.eye(s, u.shape[1]))


@pytest.mark.parametrize("dims,ranks,ok", [
    ((4, 3, 2), (2, 2, 1), True),
    ((4, 3, 2), (3, 1, 1), False),      # R_1 > R_2 R_3: subspace undetermined
    ((4, 3, 2), (5, 1, 1), False),
    ((4,), (1,), False),
    ((4, 3), (0, 1), False),
])
def test_validation(dims, ranks, ok):
    if ok:
        oracle.validate(dims, ranks, 1, 0.0)
    else:
        with pytest.raises(ValueError):
            oracle.validate(dims, ranks, 1, 0.0)


# ---------------------------------------------------------------- planted mistakes

def _pins_pass(mod):
    """Run a reduced pin set against a (possibly broken) oracle module; True if all hold."""
    try:
        x = gapped_random((6, 5, 4, 3), (3, 2, 2, 2), 7, noise=0.05)
        ranks = (3, 2, 2, 2)
        facs, _ = mod.thosvd_factors(x, ranks)
        for n in range(4):
            u, _ = svd_left(loop_unfold(x, n), ranks[n])
            if sin_theta(facs[n], u) > 1e-10:
                return False
        res = mod.hooi(x, ranks, max_iters=3)
        nx2 = float(np.sum(x * x))
        xh = einsum_reconstruct(res.core, res.factors)
        if abs(nx2 - float(np.sum(res.core ** 2)) - float(np.sum((x - xh) ** 2))) > 1e-10 * nx2:
            return False
        for k in range(1, len(res.fits)):
            if res.fits[k] < res.fits[k - 1] - 1e-13:
                return False
        cur = [f.copy() for f in facs]
        for n in range(4):
            new, _, _ = mod.hooi_update(x, cur, n, ranks[n])
            u, _ = svd_left(loop_unfold(einsum_project(x, cur, skip=n), n), ranks[n])
            if ranks[n] < x.shape[n] and sin_theta(new, u) > 1e-10:
                return False
            cur[n] = new
        return True
    except Exception:
        return False


def test_planted_mistakes_are_caught(monkeypatch):
    assert _pins_pass(hooi_ref)

    orig_lead = hooi_ref.leading_eigvecs
    orig_ttm = hooi_ref.ttm
    orig_pab = hooi_ref.project_all_but

    def smallest_first(s, r):                       # wrong end of the spectrum
        lam, v = np.linalg.eigh(s)
        return np.ascontiguousarray(v[:, :r]), lam
    monkeypatch.setattr(hooi_ref, "leading_eigvecs", smallest_first)
    assert not _pins_pass(hooi_ref)
    monkeypatch.setattr(hooi_ref, "leading_eigvecs", orig_lead)

    def ttm_untransposed(x, m, n):                  # contracts with M^T instead of M
        if m.shape[0] == x.shape[n]:
            return np.moveaxis(np.tensordot(m.T, x, axes=([1], [n])), 0, n)
        raise ValueError("shape")
    monkeypatch.setattr(hooi_ref, "ttm", ttm_untransposed)
    assert not _pins_pass(hooi_ref)
    monkeypatch.setattr(hooi_ref, "ttm", orig_ttm)

    def drop_last_mode(x, factors, skip):           # forgets one mode of the chain
        y = x
        for m, u in enumerate(factors[:-1]):
            if m != skip:
                y = orig_ttm(y, u.T, m)
        return y
    monkeypatch.setattr(hooi_ref, "project_all_but", drop_last_mode)
    assert not _pins_pass(hooi_ref)
    monkeypatch.setattr(hooi_ref, "project_all_but", orig_pab)

    def gram_of_wrong_mode(y, n):                   # wrong unfolding index
        yn = np.moveaxis(y, (n + 1) % y.ndim, 0).reshape(y.shape[(n + 1) % y.ndim], -1)
        return yn @ yn.T
    monkeypatch.setattr(hooi_ref, "gram", gram_of_wrong_mode)
    assert not _pins_pass(hooi_ref)
