"""The run driver (python -m paper_1903_02581_amd.run): its JSON-lines series
against the oracle on the 16x16 workload."""
import json

import numpy as np
import pytest

import oracle as O
from workloads import preset
from tests.gpu_util import announce, oracle_run

pytestmark = pytest.mark.gpu


def test_run_series_matches_oracle(tmp_path):
    from paper_1903_02581_amd.run import main, packet_rows
    w = preset("tiny")
    out = tmp_path / "run.jsonl"
    announce("run driver tiny 40 steps every 20")
    assert main(["--preset", "tiny", "--steps", "40", "--every", "20", "--out", str(out)]) == 0
    recs = [json.loads(x) for x in out.read_text().splitlines()]
    head, samples, tail = recs[0], recs[1:-1], recs[-1]
    assert head["run"] == "tiny" and head["points"] == w.points and head["steps"] == 40
    assert [r["step"] for r in samples] == [0, 20, 40]
    assert tail["done"] and tail["steps"] == 40 and tail["gp_steps_per_s"] > 0
    j1, j2 = packet_rows(w)
    ix = np.arange(w.nx)
    for r in samples:
        ref = O.init_state(w.psi_a, w.psi_b, w.sym) if r["step"] == 0 else oracle_run(w, r["step"])[0]
        ro = O.observables(ref, w.w_top)
        for k in ("norm", "p_tt", "p_tb", "p_bt", "p_bb", "p_b", "p_ab"):
            assert abs(r[k] - ro[k]) <= 1e-12, (r["step"], k)
        assert abs(r["entropy"] - O.entanglement(ref, ix, j1, ix, j2)) <= 1e-10
        assert r["t_fs"] == r["step"] * w.dt_fs
