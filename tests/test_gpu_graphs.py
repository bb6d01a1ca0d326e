"""Graph replay of the sweep (tucker_options.use_graphs) (needs an MI355X).

One sweep is captured as a HIP graph and replayed for every sweep.  Every replay must give what
the kernel-by-kernel launches give: the fit after every sweep, the core and the factors are
compared bitwise with an eager run of the same decomposition on the same stream, and the graph
decomposition is repeated with eager work and synchronisations in between.
"""

import numpy as np
import pytest

from synth import make_exact_rank, make_stereo_stack, make_tiny, STACK_CONFIGS

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)


def _cases():
    mini = STACK_CONFIGS["stack_mini"]
    xm = make_stereo_stack(mini["H"], mini["W"], mini["E"], mini["colorspace"], mini["seed"])
    return [
        ("stack_mini fp32", xm, mini["ranks"], 6, "fp32"),
        ("stack_mini bf16", xm, mini["ranks"], 6, "bf16"),
        ("tiny", make_tiny(0, 1e-3)[0].astype(np.float32), (16, 12, 3, 4), 5, "fp32"),
        ("order 3", make_exact_rank((90, 70, 20), (8, 6, 4), 5, 1e-3)[0].astype(np.float32), (8, 6, 4), 4, "fp32"),
    ]


def _run(x, ranks, iters, precision, graphs, stream):
    import torch
    import paper_2104_04726_amd as tk
    ctx = tk.Context(0, stream=stream, precision=precision, refine_sweeps=1, use_graphs=graphs)
    try:
        xd = torch.from_numpy(x).cuda()
        torch.cuda.synchronize()
        r = ctx.decompose(xd, ranks, iters)
        torch.cuda.synchronize()
        return (r.fit, list(r.fit_history), r.core.cpu().numpy(), [u.cpu().numpy() for u in r.factors])
    finally:
        ctx.close()


def _same(a, b):
    assert a[0] == b[0]
    assert a[1] == b[1]
    assert np.array_equal(a[2], b[2])
    for u, v in zip(a[3], b[3]):
        assert np.array_equal(u, v)


def test_graph_replays_equal_eager_sweeps():
    import torch
    st = torch.cuda.Stream()
    for name, x, ranks, iters, prec in _cases():
        _say(f"graphs vs eager: {name}")
        eager = _run(x, ranks, iters, prec, False, st)
        g1 = _run(x, ranks, iters, prec, True, st)
        _same(eager, g1)
        # eager work and synchronisations between graph decompositions, then replay again
        junk = torch.randn(1 << 20, device="cuda").sum().item()
        assert junk == junk
        g2 = _run(x, ranks, iters, prec, True, st)
        _same(eager, g2)


def test_graphs_fall_back_on_the_null_stream():
    import torch
    name, x, ranks, iters, prec = _cases()[2]
    a = _run(x, ranks, iters, prec, True, 0)          # NULL stream: sweeps launched kernel by kernel
    b = _run(x, ranks, iters, prec, False, torch.cuda.Stream())
    _same(a, b)
