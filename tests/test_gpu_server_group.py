"""Grouped served execution (needs an MI355X): requests of one shape class admitted together run their
reduced-precision sweep products as grouped persistent launches over all members' tiles.

Every product's tiles are computed by the same tile code in the same k order, whether the product is
launched alone or as part of a group, so each member's result equals the request run alone bit for
bit.  The group is forced deterministically: a large request fills the whole HBM budget while the
four group members queue behind it; when it finishes, one slot admits the first member together with
the three others of its class (they fit in the budget).
"""

import numpy as np
import pytest

from synth import make_stereo_stack, STACK_CONFIGS

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)


def _members(precision):
    c = STACK_CONFIGS["stack_mini"]
    return [dict(x=make_stereo_stack(c["H"], c["W"], c["E"], c["colorspace"], c["seed"] + 10 * k),
                 ranks=c["ranks"], iters=4, precision=precision, tag=10 + k) for k in range(4)]


def _blocker():
    c = STACK_CONFIGS["stack_mini"]
    x = make_stereo_stack(3 * c["H"], 3 * c["W"], c["E"], c["colorspace"], c["seed"] + 99)
    r = c["ranks"]
    return dict(x=x, ranks=(3 * r[0], 3 * r[1], r[2], r[3]), iters=3, precision="fp32", tag=1)


def _submit(srv, q):
    return srv.submit(q["x"], q["ranks"], q["iters"], precision=q["precision"], tag=q["tag"])


@pytest.mark.parametrize("precision", ["bf16", "fp8"])
def test_grouped_members_equal_alone(precision):
    import paper_2104_04726_amd as tk
    members, blocker = _members(precision), _blocker()
    _say(f"{precision}: members alone (1 slot, grouping off)")
    alone = {}
    with tk.Server(0, slots=1) as srv:
        for q in members:
            alone[q["tag"]] = srv.wait(_submit(srv, q), timeout=120)
        fb = srv.wait(_submit(srv, dict(blocker, iters=1)), timeout=120).footprint_bytes
    fg = alone[members[0]["tag"]].footprint_bytes
    _say(f"  footprints: member {fg}, blocker {fb}")
    assert fb >= 4 * fg, "the blocker must hold the whole budget that four members need"
    with tk.Server(0, slots=2, hbm_budget_bytes=fb, group_requests=4) as srv:
        ids = [_submit(srv, blocker)] + [_submit(srv, q) for q in members]
        res = [srv.wait(i, timeout=180) for i in ids]
        st = srv.stats()
    _say(f"  stats {st}")
    assert all(r.status == 0 for r in res), [r.error for r in res]
    assert st["grouped_requests"] == 4 and st["group_launches"] >= 1 and st["grouped_products"] >= 4
    admits = {r.tag: r.t_admit for r in res}
    assert min(admits[q["tag"]] for q in members) >= res[0].t_finish - 1e-3   # queued behind the blocker
    for q, r in zip(members, res[1:]):
        a = alone[q["tag"]]
        assert r.tag == q["tag"] and r.fit == a.fit and r.sweeps == a.sweeps
        assert np.array_equal(r.core, a.core)
        for u, v in zip(r.factors, a.factors):
            assert np.array_equal(u, v)


def test_grouping_off_and_mixed_classes_run_alone():
    import paper_2104_04726_amd as tk
    members = _members("bf16")[:2]
    other = dict(members[1], precision="fp16", tag=30)
    with tk.Server(0, slots=4, group_requests=0) as srv:
        res = [srv.wait(i, timeout=120) for i in [_submit(srv, q) for q in members]]
        st = srv.stats()
    assert all(r.status == 0 for r in res) and st["grouped_requests"] == 0
    with tk.Server(0, slots=4, group_requests=4) as srv:
        # different classes are never grouped together
        res = [srv.wait(i, timeout=120) for i in [_submit(srv, members[0]), _submit(srv, other)]]
        st = srv.stats()
    assert all(r.status == 0 for r in res) and st["grouped_requests"] == 0
