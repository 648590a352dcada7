"""Per-kernel timing through the C ABI (hrt_profile_begin / hrt_profile_end):
launch counts per kernel slot for forward, adjoint and normal calls, positive
times for every launched slot, and the record limit."""
import numpy as np
import pytest

import synth

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu


def test_profile_counts_times_and_limit():
    from paper_1604_07651_amd.hrt import Plan
    desc = synth.config_desc("c1")
    plan = Plan(desc)
    f = torch.from_numpy(synth.random_pair(desc, 5)[0].astype(np.float32)).cuda()
    print("[gpu] profile: 2 forward, 2 adjoint, 1 normal", flush=True)
    plan.profile_begin(64)
    for _ in range(2):
        g = plan.forward(f)
        plan.adjoint(g)
    plan.normal(f)
    prof = plan.profile_end()
    names = list(Plan.STAGES)
    for name in names:
        ms, n = prof[name]
        # the normal call launches no input maximum for its adjoint
        assert n == (2 if name == "adj_absmax" else 3), (name, n)
        assert ms > 0.0, name
    print("[gpu] profile: record limit", flush=True)
    plan.profile_begin(5)
    g = plan.forward(f)
    plan.adjoint(g)
    prof = plan.profile_end()
    counts = [prof[name][1] for name in names]
    assert counts == [1, 1, 1, 1, 1] + [0] * 7
    plan.close()
