"""Served execution (tucker_server_*): admission by HBM budget, concurrent requests (needs an MI355X).

* Each request's result is the same alone and in a mix of concurrent requests: every kernel's
  result depends only on its own inputs (fixed reduction orders, per-request workspaces), so the
  comparison is bitwise; results also equal a plain Context.decompose of the same request.
* Admission is first come, first served and never exceeds the budget; a request larger than the
  whole budget is refused at submit.
"""

import numpy as np
import pytest

from synth import make_exact_rank, make_stereo_stack, make_tiny, STACK_CONFIGS

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)


def _requests():
    mini, ipt = STACK_CONFIGS["stack_mini"], STACK_CONFIGS["stack_mini_ipt"]
    xm = make_stereo_stack(mini["H"], mini["W"], mini["E"], mini["colorspace"], mini["seed"])
    xi = make_stereo_stack(ipt["H"], ipt["W"], ipt["E"], ipt["colorspace"], ipt["seed"])
    xt = make_tiny(0, 1e-3)[0].astype(np.float32)
    x3 = make_exact_rank((90, 70, 20), (8, 6, 4), 5, 1e-3)[0].astype(np.float32)
    return [
        dict(x=xm, ranks=mini["ranks"], iters=6, precision="fp32", tag=1),
        dict(x=xm, ranks=mini["ranks"], iters=6, precision="bf16", tag=2),
        dict(x=xi, ranks=ipt["ranks"], iters=5, precision="fp32", tag=3),
        dict(x=xi, ranks=ipt["ranks"], iters=5, precision="fp8", tag=4),
        dict(x=xt, ranks=(16, 12, 3, 4), iters=4, precision="fp32", tag=5),
        dict(x=x3, ranks=(8, 6, 4), iters=3, precision="fp32", tag=6),
    ]


def _run(srv, reqs, together):
    out = {}
    if together:
        ids = [(q["tag"], srv.submit(q["x"], q["ranks"], q["iters"], precision=q["precision"], tag=q["tag"]))
               for q in reqs]
        for tag, rid in ids:
            out[tag] = srv.wait(rid, timeout=120)
    else:
        for q in reqs:
            rid = srv.submit(q["x"], q["ranks"], q["iters"], precision=q["precision"], tag=q["tag"])
            out[q["tag"]] = srv.wait(rid, timeout=120)
    return out


def _same(a, b):
    assert a.status == 0 and b.status == 0, (a.error, b.error)
    assert a.fit == b.fit and a.sweeps == b.sweeps
    assert np.array_equal(a.core, b.core)
    for u, v in zip(a.factors, b.factors):
        assert np.array_equal(u, v)


def test_alone_equals_mix_and_direct_decompose():
    import torch
    import paper_2104_04726_amd as tk
    reqs = _requests()
    _say("alone (1 slot, one at a time)")
    with tk.Server(0, slots=1) as srv:
        alone = _run(srv, reqs, together=False)
    _say("mix (4 slots, all submitted at once)")
    with tk.Server(0, slots=4) as srv:
        mix = _run(srv, reqs, together=True)
        st = srv.stats()
    assert st["completed"] == len(reqs) and st["failed"] == 0
    assert st["peak_running"] >= 2            # the requests really overlapped
    for q in reqs:
        _say(f"  tag {q['tag']} {q['precision']} fit {alone[q['tag']].fit:.9f}")
        _same(alone[q["tag"]], mix[q["tag"]])
    # the served result is the library's decomposition of that request
    for q in reqs:
        ctx = tk.Context(0, precision=q["precision"], refine_sweeps=1)
        try:
            r = ctx.decompose(torch.from_numpy(q["x"]).cuda(), q["ranks"], q["iters"])
        finally:
            ctx.close()
        s = alone[q["tag"]]
        assert r.fit == s.fit
        assert np.array_equal(r.core.cpu().numpy(), s.core)
        for u, v in zip(r.factors, s.factors):
            assert np.array_equal(u.cpu().numpy(), v)


def test_budget_admission_is_fifo_and_bounded():
    import paper_2104_04726_amd as tk
    reqs = _requests()[:4]
    sizes = []
    with tk.Server(0, slots=4) as probe:
        for q in reqs:
            rid = probe.submit(q["x"], q["ranks"], 1, precision=q["precision"], tag=q["tag"])
            sizes.append(probe.wait(rid, timeout=120).footprint_bytes)
    budget = int(max(sizes) * 1.2)            # room for the largest request, not for every pair
    _say(f"footprints {sizes}, budget {budget}")
    with tk.Server(0, slots=4, hbm_budget_bytes=budget) as srv:
        ids = [srv.submit(q["x"], q["ranks"], q["iters"], precision=q["precision"], tag=q["tag"]) for q in reqs]
        res = [srv.wait(i, timeout=120) for i in ids]
        st = srv.stats()
    assert all(r.status == 0 for r in res)
    assert st["peak_admitted_bytes"] <= budget
    admits = [r.t_admit for r in res]
    assert admits == sorted(admits)                       # first come, first served
    # at every admission the requests in flight (admitted, not yet finished) fit in the budget
    for r in res:
        inflight = sum(o.footprint_bytes for o in res if o.t_admit <= r.t_admit < o.t_finish)
        assert inflight <= budget


def test_refusals_and_timeouts():
    import paper_2104_04726_amd as tk
    q = _requests()[0]
    with tk.Server(0, slots=1, hbm_budget_bytes=1 << 20) as srv:
        with pytest.raises(tk.TuckerError) as e:
            srv.submit(q["x"], q["ranks"], 2)
        assert e.value.code == 2                           # ERR_OUT_OF_MEMORY: larger than the budget
    with tk.Server(0, slots=1) as srv:
        with pytest.raises(tk.TuckerError) as e:
            srv.submit(np.zeros((40, 30, 20), np.float32), (5, 5, 5), 2, precision="bf16")
        assert e.value.code == 5                           # no reduced precision for this shape
        with pytest.raises(tk.TuckerError) as e:
            srv.wait(12345, timeout=0.1)
        assert e.value.code == 1                           # unknown id
        rid = srv.submit(q["x"], q["ranks"], 30)
        with pytest.raises(tk.TuckerError) as e:
            srv.wait(rid, timeout=0.0)
        assert e.value.code == 6                           # not finished yet
        assert srv.wait(rid, timeout=120).status == 0
