"""The autotuner (needs an MI355X): with tucker_options.autotune the first decomposition of a shape
times the candidate launch choices (FP32 product tile shape, FP64 Gram split count) and keeps the
fastest; later decompositions of that shape, tuned or not, reuse the kept choices, so their results are
bit-for-bit those of the tuned run, and they still match the oracle."""

import numpy as np
import pytest

import oracle
from synth import make_stereo_stack, STACK_CONFIGS

pytestmark = pytest.mark.gpu


def _dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).cuda()


def test_autotune_times_new_shapes_and_keeps_choices():
    import paper_2104_04726_amd as tk
    c = STACK_CONFIGS["stack_mini"]
    # a shape no other test uses, so that its keys are new in this process
    x32 = make_stereo_stack(c["H"] + 8, c["W"] + 16, c["E"], c["colorspace"], c["seed"] + 100)
    ranks = c["ranks"]
    before = tk.autotune_table()
    with tk.Context(0, autotune=True) as ctx:
        a = ctx.decompose(_dev(x32), ranks, 3)
    table = tk.autotune_table()
    new = [ln for ln in table.splitlines() if ln not in before.splitlines()]
    print("\n".join(new), flush=True)
    timed = [ln for ln in new if "(heuristic)" not in ln]
    assert any(ln.startswith("op 1 ") for ln in timed), new      # FP32 product tiles
    assert any(ln.startswith("op 2 ") for ln in timed), new      # FP64 Gram splits
    for ln in timed:
        ms = [float(v) for v in ln.split(" ms ")[1].split()]
        assert all(m > 0 for m in ms), ln
    with tk.Context(0) as ctx:
        b = ctx.decompose(_dev(x32), ranks, 3)
    assert a.fit == b.fit
    assert np.array_equal(a.core.cpu().numpy(), b.core.cpu().numpy())
    for u, v in zip(a.factors, b.factors):
        assert np.array_equal(u.cpu().numpy(), v.cpu().numpy())
    assert tk.autotune_table() == table          # nothing new: every key was already fixed
    o = oracle.hooi(x32.astype(np.float64), ranks, 3)
    m = oracle.compare(dict(core=a.core.cpu().numpy(), factors=[u.cpu().numpy() for u in a.factors], fit=a.fit),
                       dict(core=o.core, factors=o.factors, fit=o.fits[-1]))
    assert m["fit"] <= 1e-5 and m["core_norm"] <= 1e-5
