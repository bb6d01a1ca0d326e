"""Pins of the oracle's pairwise-perturbation HOOI (oracle/pp_ref.py) -- CPU only.

* eq. (11) is the first-order part of the multilinear expansion of eq. (9): for an order-3 tensor the
  remainder Y(n) - Y~(n) is exactly the one second-order term X x_i dS(i)^T x_j dS(j)^T (written out
  with einsum), for any dS; for order 4 it is second order (halving dS divides it by 4 as dS -> 0);
  with dS = 0 the approximation is exact;
* the operators of eq. (12)-(13) equal X projected on all modes but one (or two), written with einsum;
* the Procrustes representative spans the same subspace, recovers the reference from any rotated
  copy of it, and is no farther from the reference than randomly rotated bases;
* pp_tol = 0 never switches and gives plain HOOI; on gapped inputs the switching run converges to
  plain HOOI's fit;
and planted mistakes in source copies of the module fail these checks.
"""

import inspect
import math

import numpy as np
import pytest

import oracle
from oracle import pp_ref
from synth import make_exact_rank
from test_oracle_pins import einsum_project, sin_theta


def _orth(rng, s, r):
    return np.linalg.qr(rng.standard_normal((s, r)))[0]


def _exact_y(x, factors, n):
    return einsum_project(x, factors, skip=n)


def _order3_identity_ok(mod, seed=1, tol=1e-12):
    rng = np.random.default_rng(seed)
    x = rng.standard_normal((7, 6, 5))
    ranks = (3, 2, 4)
    ref = [_orth(rng, s, r) for s, r in zip(x.shape, ranks)]
    cur = [u + 0.3 * rng.standard_normal(u.shape) for u in ref]
    single, pair = mod.pp_operators(x, ref)
    for n in range(3):
        i, j = [m for m in range(3) if m != n]
        approx = mod.pp_tensor(single, pair, cur, ref, n)
        exact = _exact_y(x, cur, n)
        d = [None] * 3
        d[i], d[j] = (cur[i] - ref[i]), (cur[j] - ref[j])
        letters = "abc"
        out = "".join(letters[m] if m == n else "ijk"[m] for m in range(3))
        second = np.einsum(f"abc,{letters[i]}{'ijk'[i]},{letters[j]}{'ijk'[j]}->{out}", x, d[i], d[j])
        if np.max(np.abs(exact - approx - second)) > tol * np.max(np.abs(exact)):
            return False
    return True


def test_first_order_remainder_is_the_second_order_term():
    assert _order3_identity_ok(pp_ref)


def test_order4_remainder_is_second_order_and_exact_at_reference():
    rng = np.random.default_rng(2)
    x = rng.standard_normal((6, 5, 4, 3))
    ranks = (3, 3, 2, 2)
    ref = [_orth(rng, s, r) for s, r in zip(x.shape, ranks)]
    d = [rng.standard_normal(u.shape) for u in ref]
    single, pair = pp_ref.pp_operators(x, ref)
    for n in range(4):
        assert np.max(np.abs(pp_ref.pp_tensor(single, pair, ref, ref, n) - _exact_y(x, ref, n))) <= 1e-13
        errs = []
        for t in (1e-2, 5e-3):
            cur = [u + t * e for u, e in zip(ref, d)]
            errs.append(np.linalg.norm(_exact_y(x, cur, n) - pp_ref.pp_tensor(single, pair, cur, ref, n)))
        assert abs(errs[0] / errs[1] - 4.0) <= 0.1, errs


def test_operators_are_the_partial_projections():
    rng = np.random.default_rng(3)
    x = rng.standard_normal((5, 4, 6, 3))
    ref = [_orth(rng, s, r) for s, r in zip(x.shape, (2, 3, 2, 2))]
    single, pair = pp_ref.pp_operators(x, ref)
    for n in range(4):
        assert np.max(np.abs(single[n] - einsum_project(x, ref, skip=n))) <= 1e-13
    for (i, n), y in pair.items():
        fs = [u if m not in (i, n) else np.eye(x.shape[m]) for m, u in enumerate(ref)]
        assert np.max(np.abs(y - einsum_project(x, fs))) <= 1e-13


def test_procrustes_representative():
    rng = np.random.default_rng(4)
    ref = _orth(rng, 12, 5)
    q = _orth(rng, 5, 5)
    assert np.max(np.abs(pp_ref.procrustes_align(ref @ q, ref) - ref)) <= 1e-13
    u = _orth(rng, 12, 5)
    a = pp_ref.procrustes_align(u, ref)
    assert sin_theta(a, u) <= 1e-13 and sin_theta(u, a) <= 1e-13
    assert np.linalg.norm(a.T @ a - np.eye(5)) <= 1e-13
    best = np.linalg.norm(a - ref)
    for _ in range(50):
        assert best <= np.linalg.norm(u @ _orth(rng, 5, 5) - ref) + 1e-12


def test_pp_tol_zero_is_plain_hooi():
    x, _, _ = make_exact_rank((14, 12, 3, 5), (5, 4, 3, 3), 5, 0.1)
    ranks = (5, 4, 3, 3)
    r = pp_ref.hooi_pp(x, ranks, 6, pp_tol=0.0)
    h = oracle.hooi(x, ranks, 6)
    assert r.kinds == ["als"] * 6
    assert r.fits == h.fits
    for a, b in zip(r.factors, h.factors):
        assert np.array_equal(a, b)


def test_subspace_distance_is_the_rms_sine():
    rng = np.random.default_rng(6)
    thetas = np.array([0.3, 0.01, 0.7])
    q, _ = np.linalg.qr(rng.standard_normal((9, 6)))
    u = q[:, :3]
    v = q[:, :3] * np.cos(thetas) + q[:, 3:] * np.sin(thetas)
    assert abs(pp_ref.subspace_distance(u, v) - math.sqrt(np.mean(np.sin(thetas) ** 2))) <= 1e-14
    assert pp_ref.subspace_distance(u, u @ _orth(rng, 3, 3)) <= 1e-14


def test_switching_run_reaches_the_plain_hooi_fit():
    x, _, _ = make_exact_rank((30, 28, 3, 6), (8, 7, 3, 4), 1, 0.05)
    ranks = (8, 7, 3, 4)
    r = pp_ref.hooi_pp(x, ranks, 12, pp_tol=0.1)
    h = oracle.hooi(x, ranks, 12)
    assert "pp" in r.kinds and r.kinds[0] == "als"
    assert abs(r.fit - h.fits[-1]) <= 1e-10
    nx2 = float(np.sum(x * x))
    assert abs(r.fit - (1 - math.sqrt(max(nx2 - float(np.sum(r.core ** 2)), 0)) / math.sqrt(nx2))) <= 1e-13
    for a, b in zip(r.factors, h.factors):
        assert sin_theta(a, b) <= 1e-6


# ---------------------------------------------------------------- planted mistakes

def _mutant(old, new):
    src = inspect.getsource(pp_ref)
    assert src.count(old) == 1, old
    ns = {"__name__": "oracle.pp_mutant", "__package__": "oracle"}
    exec(compile(src.replace(old, new), "pp_mutant", "exec"), ns)

    class M:
        pass
    m = M()
    for k in ("pp_operators", "pp_tensor", "procrustes_align"):
        setattr(m, k, ns[k])
    return m


@pytest.mark.parametrize("old,new", [
    ("ds = factors[i] - ref[i]", "ds = factors[i]"),                              # the factor, not the change
    ("y = y + ttm(pair[(min(i, n), max(i, n))], ds.T, i)",
     "y = y + ttm(pair[(min(i, n), max(i, n))], ds.T, i) if i != len(factors) - 1 else y"),   # a dropped term
    ("if j not in (i, n):", "if j != i:"),                                       # operator contracts mode n too
    ("y = y + ttm(pair[(min(i, n), max(i, n))], ds.T, i)",
     "y = y - ttm(pair[(min(i, n), max(i, n))], ds.T, i)"),                      # wrong sign
])
def test_planted_mistakes_are_caught(old, new):
    assert _order3_identity_ok(pp_ref)
    try:
        ok = _order3_identity_ok(_mutant(old, new))
    except Exception:
        ok = False
    assert not ok
