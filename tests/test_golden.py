"""Stored fixtures: the paper's Table I parameters (cited in the file) and a
snapshot of the oracle written by tests/golden/make_oracle_golden.py."""
import json
import math
import os

import numpy as np

from paper_2406_01713_amd import scenes as S

GOLD = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def test_rr_scene_uses_table1_goal():
    t = json.load(open(os.path.join(GOLD, "table1_rr.json")))
    s = S.scene_c1()
    assert np.allclose(s["goal_c"], t["q_goal"])
    # the configuration box of the 2-D workload contains Table I's start and goal
    assert all(-math.pi <= v <= math.pi for v in t["q_start"] + t["q_goal"])


def test_oracle_matches_its_stored_snapshot(oracle):
    import importlib.util
    spec = importlib.util.spec_from_file_location("mk", os.path.join(GOLD, "make_oracle_golden.py"))
    mk = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mk)
    gold = json.load(open(os.path.join(GOLD, "oracle_small.json")))
    for name, s in mk.cases():
        u, g, st, dq = oracle.estimate(s, dq=True)
        ref = gold[name]
        # libm may pick different code paths on another host CPU: last-bit slack
        assert np.allclose(u, np.array(ref["u"]), rtol=1e-10, atol=1e-15), name
        assert np.allclose(g, np.array(ref["grad"]), rtol=1e-10, atol=1e-15), name
        assert np.allclose(st, np.array(ref["stats"]), rtol=1e-8, atol=1e-15), name
        assert np.allclose(dq, np.array(ref["dq"]), rtol=1e-10, atol=1e-15), name
