"""Walk-level parity bars shared by the GPU tests.

The GPU and the oracle draw every walk from the same Philox counters, so a
walk takes the same steps on both sides unless rounding moves a decision (an
eps-shell test, the nearest component) the other way; from then on the two
walks differ.  Measured on MI355X, 127 or 128 of every 128 walks keep the same
step count in FP32 (all of them in FP64) on the 2- to 8-D scenes, so the bars
sit a few walks below that."""

WALK_MATCH_FP64 = 0.98
WALK_MATCH_FP32 = 0.95


def walk_match(fp64):
    return WALK_MATCH_FP64 if fp64 else WALK_MATCH_FP32


def check_rate(what, fp64, same, total):
    rate = same / total
    print(f"{what} {'fp64' if fp64 else 'fp32'}: {same}/{total} walks step for step ({rate:.3f})")
    assert rate >= walk_match(fp64), (what, rate)
