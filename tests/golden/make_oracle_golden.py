"""Writes oracle_small.json: FP64 oracle outputs on small fixed cases.

Calls only the oracle (and the seeded scene generators).  Re-run only when the
oracle's arithmetic changes for a reason that a passage of the paper, or a
stated reading of it, justifies."""
import json
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import oracle as O  # noqa: E402
from paper_2406_01713_amd import scenes as S  # noqa: E402


def cases():
    c1 = S.scene_c1(n_walks=256, seed=3)
    c1["queries"] = c1["queries"][::7]
    yield "c1_every7th_n256", c1
    c3 = S.scene_c3(n_walks=64, seed=5)
    c3["queries"] = c3["queries"][::128]
    yield "c3_every128th_n64", c3
    b = S.scene_ball(5, R=1.0, sigma=2.0, eps=1e-4,
                     queries=np.array([[0.3, 0.1, 0, 0, 0], [0, 0, 0.6, 0, 0]]), n_walks=128, seed=1)
    yield "ball_d5_sigma2_n128", b


def main():
    out = {}
    for name, s in cases():
        u, g, st, dq = O.estimate(s, dq=True)
        out[name] = {"u": u.tolist(), "grad": g.tolist(), "stats": st.tolist(), "dq": dq.tolist()}
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "oracle_small.json")
    with open(path, "w") as f:
        json.dump(out, f, indent=1)
    print("wrote", path)


if __name__ == "__main__":
    main()
