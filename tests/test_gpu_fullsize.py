"""Full-size checks at the benchmark's own configuration (needs an MI355X).

The 1080p stack (1080x1920x3x14, ranks 256/384/3/8, 20 sweeps) and the 4K stack
(2160x3840x3x10 IPT, ranks 512/768/3/6, 15 sweeps) are decomposed with the options bench.py
uses.  Their results are checked against:

* the FP64 oracle's stored trajectory for the same seeded tensor (tests/golden/*_oracle.json,
  written by tests/golden/make_stack_oracle.py, which calls only the oracle): the final fit and
  the core norm to 1e-5 (FP32) or 1e-3 (BF16 + FP32 refinement); the per-sweep fit (from
  ||X||^2 - ||G||^2 with the FP32 core) within the FP32 error of ||G||^2 amplified by the
  cancellation in that difference;
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


def _decompose(name, precision="fp32"):
    import torch
    import paper_2104_04726_amd as tk
    c = STACK_CONFIGS[name]
    x32 = _stack(name)
    ctx = tk.Context(0, precision=precision, refine_sweeps=1)
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
