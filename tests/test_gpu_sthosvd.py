"""The sequentially truncated ("interlaced") HOSVD start on the GPU against the oracle's
(needs an MI355X).  Sec. III-B.1 offers it as the cheaper start: each mode's factor from the
Gram of the tensor already projected on the earlier modes' factors.  Comparisons as in
test_gpu_hooi.py: strict 1e-5 parity on gapped exact-rank inputs; on image stacks the second-order
quantities at 1e-5 and the reconstruction within the subspace-iteration allowance, with the
oracle's converged leading eigenvectors inside the GPU subspaces.
"""

import numpy as np
import pytest

import oracle
from synth import make_exact_rank, make_stereo_stack, make_tiny, STACK_CONFIGS
from test_gpu_hooi import INIT_ITERS, _check_strict, _dev, _gpu, _ora, _say, _stack_checks

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import paper_2104_04726_amd as tk
    c = tk.Context(0, start="sthosvd")
    yield c
    c.close()


@pytest.mark.parametrize("iters", [0, 3])
def test_tiny_sthosvd_matches_oracle(ctx, iters):
    x, _, _ = make_tiny(0, 1e-3)
    x32 = x.astype(np.float32)
    _say(f"tiny sthosvd iters={iters}")
    g = _gpu(ctx, x32, (16, 12, 3, 4), iters)
    o = _ora(x32, (16, 12, 3, 4), iters, start="sthosvd")
    _check_strict(oracle.compare(g, o))


@pytest.mark.parametrize("dims,ranks", [((40, 36, 30), (6, 5, 4)), ((20, 18, 6, 5, 4), (4, 3, 2, 2, 2)),
                                        ((90, 70, 3, 6), (12, 10, 3, 4))])
def test_exact_rank_sthosvd_equals_generating_subspaces(ctx, dims, ranks):
    x, _, facs = make_exact_rank(dims, ranks, seed=3, noise_rel=1e-4)
    x32 = x.astype(np.float32)
    _say(f"exact rank sthosvd {dims}")
    g = _gpu(ctx, x32, ranks, 0)
    o = _ora(x32, ranks, 0, start="sthosvd")
    _check_strict(oracle.compare(g, o))
    for u, t in zip(g["factors"], facs):
        assert np.linalg.norm(u - t @ (t.T @ u), 2) <= 1e-3     # noise 1e-4: Wedin's bound


@pytest.mark.parametrize("name", ["stack_mini", "stack_mini_ipt"])
@pytest.mark.parametrize("sweeps", [0, "all"])
def test_stack_sthosvd_matches_oracle(ctx, name, sweeps):
    c = STACK_CONFIGS[name]
    x32 = make_stereo_stack(c["H"], c["W"], c["E"], c["colorspace"], c["seed"])
    ranks = c["ranks"]
    iters = c["sweeps"] if sweeps == "all" else sweeps
    _say(f"stack {name} sthosvd, {iters} sweeps")
    g = _gpu(ctx, x32, ranks, iters)
    o = _ora(x32, ranks, iters, start="sthosvd")
    _stack_checks(x32, ranks, g, o, INIT_ITERS + iters, f"{name} sthosvd")


def test_stack1080_sthosvd_start_matches_oracle(ctx):
    """The 1080p stack's ST-HOSVD start (max_iters = 0) against the oracle's, plus the exact error
    identity of the sequentially truncated HOSVD evaluated from the GPU's own spectra bound."""
    c = STACK_CONFIGS["stack1080"]
    x32 = make_stereo_stack(c["H"], c["W"], c["E"], c["colorspace"], c["seed"])
    ranks = c["ranks"]
    _say("stack1080 sthosvd start")
    g = _gpu(ctx, x32, ranks, 0)
    o = _ora(x32, ranks, 0, start="sthosvd")
    _stack_checks(x32, ranks, g, o, INIT_ITERS, "stack1080 sthosvd")
    # the start is at least as good as the bound sum_n tau_n^2 of the T-HOSVD says
    th = oracle.hooi(x32.astype(np.float64), ranks, 0)
    nx = float(np.linalg.norm(x32.astype(np.float64)))
    tau2 = sum(float(np.sum(lam[r:])) for lam, r in zip(th.spectra, ranks))
    assert (1.0 - g["fit"]) * nx <= np.sqrt(tau2) * (1 + 1e-5)
    _say(f"  GPU start time {g['stats']['init_ms']:.2f} ms")
