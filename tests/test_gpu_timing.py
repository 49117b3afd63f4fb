"""Per-pass kernel timing (measurement API): launch counts per pass kind follow
the pass plans, durations are positive, and timing leaves the state unchanged."""
import numpy as np
import pytest

from workloads import preset
from tests.gpu_util import announce

pytestmark = pytest.mark.gpu


# 1100 four-pass steps record 4402 launches: past the 4096 event pairs of the pool,
# so the pending pairs are folded into the sums once mid-call
@pytest.mark.parametrize("name,plan,n", [("tiny", 0, 7), ("tiny", 1, 7), ("diff", 0, 7), ("tiny", 1, 1100)])
def test_pass_timing_counts_and_no_side_effect(name, plan, n):
    from paper_1903_02581_amd import Propagator
    w = preset(name)
    announce(f"pass timing {name} plan={plan} steps={n}")
    ref = Propagator.from_workload(w)
    ref.set_pass_plan(plan)
    ref.step(n)
    want = ref.store_state()
    ref.close()
    p = Propagator.from_workload(w)
    p.set_pass_plan(plan)
    p.pass_timing(True)
    p.step(n)
    t = p.pass_times()
    p.pass_timing(False)
    assert np.array_equal(p.store_state(), want)
    counts = {k: c for k, (_, c) in t.items()}
    if p.passes_per_step == 3:
        # x1 opens and closes with half steps and merges in between; the x2 half that
        # closes the call runs as a line pass
        assert counts == {"x1": n + 1, "plane": n, "y1": n, "x2": 1}
    else:
        assert counts == {"x1": n + 1, "x2": n + 1, "y1": n, "y2": n}
    assert all(sec > 0.0 for sec, _ in t.values())
    assert p.pass_times() == t                # reading does not reset the sums
    p.pass_timing(True)                       # a new recording starts empty
    assert p.pass_times() == {}
    p.close()
