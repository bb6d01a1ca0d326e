"""Full-size checks at the benchmark's own configuration (needs an MI355X).

The 1080p stack (1080x1920x3x14, ranks 256/384/3/8, 20 sweeps) and the 4K stack
(2160x3840x3x10 IPT, ranks 512/768/3/6, 15 sweeps) are decomposed with the options bench.py
uses.  Their results are checked against:

* the FP64 oracle's stored trajectory for the same seeded tensor (tests/golden/*_oracle.json,
  written by tests/golden/make_stack_oracle.py, which calls only the oracle): the final fit and
  the core norm to 1e-5 (FP32) or 1e-3 (BF16 + FP32 refinement); the per-sweep fit (from
  ||X||^2 - ||G||^2 with the FP32 core) within the FP32 error of ||G||^2 amplified by the
  cancellation in that difference;
* the FP64 oracle run live on the host for the 1080p stack (T-HOSVD + 20 sweeps, about 20 s, and one
  more sweep for the precision variants): the reconstruction through the rotation-invariant
  core-space difference, within 1e-5 plus the subspace-iteration allowance of tests/allowances.py
  (FP32), or within 1e-3 plus one boundary direction pair per degenerate mode (BF16, FP16, FP8
  after their FP32 refinement sweep); fit and core norm to 1e-5 (FP32) or 1e-3;
* properties that hold at any size, evaluated on the host in FP64 from the GPU's own outputs:
  orthonormal factors, the identity fit = 1 - sqrt(||X||^2 - ||G||^2) / ||X|| for orthonormal
  factors (within the same cancellation bound), a fit history that never decreases by more than
  that bound, and sampled core entries against
  their definition G = X x_1 U_1^T ... x_4 U_4^T with Higham's a-priori bound for the FP32 chain.
"""

import json
import math
import os

import numpy as np
import pytest

import oracle
from allowances import leading_containment, pair_allowance, si_allowance
from synth import STACK_CONFIGS, make_stereo_stack

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
U32 = 2.0 ** -24


def _say(msg):
    print(msg, flush=True)


def _golden(name):
    path = os.path.join(GOLDEN, f"{name}_oracle.json")
    if not os.path.exists(path):
        pytest.skip(f"{path} not generated")
    return json.load(open(path))


_CACHE = {}


def _stack(name):
    if name not in _CACHE:
        c = STACK_CONFIGS[name]
        _say(f"generating {name}")
        _CACHE[name] = make_stereo_stack(c["H"], c["W"], c["E"], c["colorspace"], c["seed"])
    return _CACHE[name]


def _decompose(name, precision="fp32", **kw):
    import torch
    import paper_2104_04726_amd as tk
    c = STACK_CONFIGS[name]
    x32 = _stack(name)
    ctx = tk.Context(0, precision=precision, refine_sweeps=1, **kw)
    try:
        _say(f"decomposing {name} {precision}")
        res = ctx.decompose(torch.from_numpy(x32).cuda(), c["ranks"], c["sweeps"])
    finally:
        ctx.close()
    core = res.core.cpu().numpy().astype(np.float64)
    factors = [u.cpu().numpy().astype(np.float64) for u in res.factors]
    return x32, res, core, factors


def _core_entries(x32, factors, idx):
    """G[r0, r1, r2, r3] and the bound term (|X| x |U|^T) for sampled entries, in FP64."""
    x = x32.astype(np.float64)
    ax = np.abs(x)
    vals, absv = [], []
    for (a, b, c, d) in idx:
        w = np.outer(factors[2][:, c], factors[3][:, d])            # (3, I)
        m = np.tensordot(x, w, axes=([2, 3], [0, 1]))                # (H, W)
        vals.append(factors[0][:, a] @ m @ factors[1][:, b])
        aw = np.abs(w)
        am = np.tensordot(ax, aw, axes=([2, 3], [0, 1]))
        absv.append(np.abs(factors[0][:, a]) @ am @ np.abs(factors[1][:, b]))
    return np.array(vals), np.array(absv)


def _properties(x32, res, core, factors, fit_tol, hist_slack):
    for u in factors:
        e = np.linalg.norm(u.T @ u - np.eye(u.shape[1]), 2)
        assert e <= 1e-5, e
    nx2 = float(np.sum(x32.astype(np.float64) ** 2))
    ng2 = float(np.sum(core * core))
    fit_id = 1.0 - math.sqrt(max(nx2 - ng2, 0.0)) / math.sqrt(nx2)
    assert abs(fit_id - res.fit) <= fit_tol, (fit_id, res.fit)
    h = res.fit_history
    assert all(b >= a - hist_slack for a, b in zip(h, h[1:])), h
    rng = np.random.default_rng(7)
    R = core.shape
    idx = [(0, 0, 0, 0)] + [tuple(int(rng.integers(0, r)) for r in R) for _ in range(5)]
    ref, absr = _core_entries(x32, factors, idx)
    got = np.array([core[i] for i in idx])
    K = sum(x32.shape)
    assert np.all(np.abs(got - ref) <= 4 * K * U32 * absr + 1e-7 * np.abs(ref)), (got, ref)


@pytest.mark.parametrize("name", ["stack1080", "stack2160"])
def test_fp32_matches_stored_oracle_and_properties(name):
    g = _golden(name)
    x32, res, core, factors = _decompose(name)
    _say(f"  fit {res.fit:.10f} oracle {g['fits'][-1]:.10f}")
    assert abs(res.fit - g["fits"][-1]) <= 1e-5
    assert len(res.fit_history) == len(g["fits"])
    # the per-sweep fit is 1 - sqrt(||X||^2 - ||G||^2) / ||X|| with the FP32 core: a relative
    # error e of ||G||^2 (FP32 accumulation along the product chain, e <= (sum s_n) u) is
    # amplified by the cancellation to about e ||G||^2 / (2 ||X|| ||X - Xhat||); the returned fit
    # is the explicit residual and is binding above
    nx2 = g["x_norm2"]
    resid = (1.0 - g["fits"][-1]) * math.sqrt(nx2)
    amp = g["core_norm"] ** 2 / (2.0 * math.sqrt(nx2) * resid)
    tol_hist = max(1e-5, 2.0 * sum(x32.shape) * U32 * amp * (1.0 - g["fits"][-1]))
    dev = [abs(a - b) for a, b in zip(res.fit_history, g["fits"])]
    _say(f"  per-sweep fit deviation {['%.1e' % d for d in dev]} (bound {tol_hist:.1e})")
    assert max(dev) <= tol_hist
    assert abs(np.linalg.norm(core) - g["core_norm"]) <= 1e-5 * g["core_norm"]
    _properties(x32, res, core, factors, tol_hist, tol_hist)


@pytest.mark.parametrize("name", ["stack1080", "stack2160"])
def test_bf16_then_refine_matches_stored_oracle(name):
    g = _golden(name)
    x32, res, core, factors = _decompose(name, "bf16")
    _say(f"  fit {res.fit:.10f} oracle {g['fits'][-1]:.10f}")
    assert abs(res.fit - g["fits"][-1]) <= 1e-3
    assert abs(np.linalg.norm(core) - g["core_norm"]) <= 1e-3 * g["core_norm"]
    for u in factors:
        assert np.linalg.norm(u.T @ u - np.eye(u.shape[1]), 2) <= 1e-5


def test_exact_fit_history_with_tolerance_is_monotone():
    """With tol > 0 every sweep's fit is the explicit residual: it never decreases (slack 1e-6)
    and the stop happens once consecutive fits differ by less than tol."""
    import torch
    import paper_2104_04726_amd as tk
    c = STACK_CONFIGS["stack1080"]
    x32 = _stack("stack1080")
    ctx = tk.Context(0)
    try:
        res = ctx.decompose(torch.from_numpy(x32).cuda(), c["ranks"], 20, tol=1e-9)
    finally:
        ctx.close()
    h = res.fit_history
    _say(f"  exact history {['%.9f' % f for f in h]}")
    assert all(b >= a - 1e-6 for a, b in zip(h, h[1:])), h
    assert abs(h[-1] - res.fit) <= 1e-7
    if res.sweeps < 20:
        assert abs(h[-1] - h[-2]) < 1e-9
    g = _golden("stack1080")
    assert abs(res.fit - g["fits"][res.sweeps]) <= 1e-5


# ------------------------------------------------------------------ live oracle at 1080p

@pytest.fixture(scope="module")
def oracle1080():
    """The FP64 oracle on the 1080p stack: 20 sweeps (the FP32 run) and one more, resumed from
    them (the reduced-precision runs end with an FP32 refinement sweep: 20 + 1)."""
    import time
    c = STACK_CONFIGS["stack1080"]
    x = _stack("stack1080").astype(np.float64)
    t = time.perf_counter()
    _say("oracle: stack1080, T-HOSVD + 20 sweeps")
    o20 = oracle.hooi(x, c["ranks"], 20)
    _say(f"  {time.perf_counter() - t:.1f} s, fit {o20.fits[-1]:.10f}; one more sweep")
    o21 = oracle.hooi(x, c["ranks"], 1, init=o20.factors)
    _say(f"  fit {o21.fits[-1]:.10f}")
    del x
    return o20, o21


def _as_dict(res, core, factors):
    return dict(core=core, factors=factors, fit=res.fit)


def test_fp32_1080_matches_live_oracle(oracle1080):
    o, _ = oracle1080
    c = STACK_CONFIGS["stack1080"]
    x32, res, core, factors = _decompose("stack1080")
    m = oracle.compare(_as_dict(res, core, factors), dict(core=o.core, factors=o.factors, fit=o.fits[-1]))
    steps = 20 + c["sweeps"]          # cold-start steps + one warm step per sweep
    recon_tol = 1e-5 + si_allowance(o.spectra, x32.shape, c["ranks"], steps)
    _say(f"  fp32: fit {m['fit']:.2e} rho {m['rho']:.2e} core {m['core_norm']:.2e} recon {m['recon']:.2e} "
         f"(bound {recon_tol:.2e}) sin {['%.2e' % v for v in m['sin_theta']]}")
    assert m["fit"] <= 1e-5 and m["rho"] <= 1e-5 and m["core_norm"] <= 1e-5, m
    assert m["recon"] <= recon_tol
    for n in (0, 1):
        k, sine, bound = leading_containment(o.factors[n], factors[n], o.spectra[n], steps)
        _say(f"    mode {n + 1}: leading {k} directions contained to {sine:.2e} (bound {bound + 1e-5:.2e})")
        assert k >= 1 and sine <= bound + 1e-5
    assert m["sin_theta"][2] <= 1e-5                     # R3 = s3: the whole space
    k, sine, bound = leading_containment(o.factors[3], factors[3], o.spectra[3], resid=0.0)
    _say(f"    mode 4: leading {k} directions contained to {sine:.2e} (bound {bound + 1e-5:.2e})")
    assert k >= 1 and sine <= bound + 1e-5


@pytest.mark.parametrize("prec", ["bf16", "fp16", "fp8"])
def test_lowp_1080_matches_live_oracle(oracle1080, prec):
    """The precision variants: 20 sweeps with BF16 / FP16 / FP8 contractions, then one FP32
    refinement sweep, against the oracle's 21 sweeps: reconstruction <= 1e-3 (plus one boundary
    direction pair per degenerate mode), fit and core norm <= 1e-3."""
    _, o = oracle1080
    c = STACK_CONFIGS["stack1080"]
    x32, res, core, factors = _decompose("stack1080", prec)
    assert res.sweeps == c["sweeps"] and res.stats["refine_sweeps"] == 1
    m = oracle.compare(_as_dict(res, core, factors), dict(core=o.core, factors=o.factors, fit=o.fits[-1]))
    tol = 1e-3 + pair_allowance(o.spectra, c["ranks"])
    _say(f"  {prec}: fit {m['fit']:.2e} core {m['core_norm']:.2e} recon {m['recon']:.2e} (bound {tol:.2e}) "
         f"sin {['%.2e' % v for v in m['sin_theta']]}")
    assert m["recon"] <= tol, m
    assert m["fit"] <= 1e-3 and m["core_norm"] <= 1e-3, m
    for u in factors:
        assert np.linalg.norm(u.T @ u - np.eye(u.shape[1]), 2) <= 1e-5
