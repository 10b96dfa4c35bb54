"""Host-side checks of the obstacle clusters the walk kernels cull with (no
GPU): the cluster order is a permutation with padding only at the end, every
member lies inside its cluster's bounding sphere, and the culling test
|x - C| (1 - m) - rho' never exceeds a member's distance as the kernels
compute it (emulated here operation by operation in the table's precision)."""
import numpy as np
import pytest

from paper_2406_01713_amd import scenes as S

CL = 8


@pytest.fixture(scope="module")
def B():
    from paper_2406_01713_amd import binding
    return binding


def _sets():
    c3 = S.scene_c3(n_walks=16)
    c5 = S.scene_c5(n_starts=4, n_walks=16)
    big = S.scene_c4_env(5, n_walks=16, q_cap=4)
    return [("c3", c3), ("c5", c5), (big["name"], big)]


@pytest.mark.parametrize("fp64", [False, True])
def test_cluster_order_is_a_padded_permutation(B, fp64):
    assert CL == B.WOS_CLUSTER_ROWS
    for name, s in _sets():
        out = B.wos_debug_clusters(s["d"], s["sph_c"], s["sph_r"], s["box_c"], s["box_h"], fp64=fp64)
        for kind, n in (("sph", len(s["sph_r"])), ("box", len(s["box_c"]))):
            order, bnd = out[kind]
            if n < 64:
                assert len(order) == 0 and len(bnd) == 0
                continue
            n_cl = -(-n // CL)
            assert len(order) == n_cl * CL and bnd.shape == (n_cl, s["d"] + 1)
            assert np.array_equal(np.sort(order[:n]), np.arange(n)), name
            assert np.all(order[n:] == -1), name


def test_small_sets_are_not_clustered(B):
    rng = np.random.default_rng(0)
    for n in (0, 1, 63):
        out = B.wos_debug_clusters(3, rng.normal(size=(n, 3)), rng.uniform(0.1, 0.2, n))
        assert len(out["sph"][0]) == 0
    out = B.wos_debug_clusters(3, rng.normal(size=(64, 3)), rng.uniform(0.1, 0.2, 64))
    assert len(out["sph"][0]) == 64


def _rounded(a, fp64):
    return np.asarray(a, np.float64) if fp64 else np.asarray(a, np.float32).astype(np.float64)


@pytest.mark.parametrize("fp64", [False, True])
def test_members_inside_bounds(B, fp64):
    """rho' >= (|c_j - C| + r_j) (1 + 2^-15 in FP32) for every member, in FP64
    on the values the device tables hold (boxes: r_j = |h_j|)."""
    rel = 2.0 ** -44 if fp64 else 2.0 ** -15
    for name, s in _sets():
        out = B.wos_debug_clusters(s["d"], s["sph_c"], s["sph_r"], s["box_c"], s["box_h"], fp64=fp64)
        for kind in ("sph", "box"):
            order, bnd = out[kind]
            if len(order) == 0:
                continue
            if kind == "sph":
                c, rad = _rounded(s["sph_c"], fp64), _rounded(s["sph_r"], fp64)
            else:
                c = _rounded(s["box_c"], fp64)
                rad = np.sqrt((_rounded(s["box_h"], fp64) ** 2).sum(1))
            for g in range(len(bnd)):
                m = order[g * CL:(g + 1) * CL]
                m = m[m >= 0]
                need = np.linalg.norm(c[m] - bnd[g, :-1], axis=1) + rad[m]
                assert np.all(bnd[g, -1] >= need.max() * (1 + rel)), (name, kind, g)


def _f32_sqdist(x, c):
    """FP32 sum of squared differences as the kernels form it: first product,
    then fused multiply-adds (each rounded once to FP32)."""
    t = (x[:, None, 0] - c[None, :, 0]).astype(np.float32)
    acc = (t * t).astype(np.float32)
    for i in range(1, x.shape[1]):
        t = (x[:, None, i] - c[None, :, i]).astype(np.float32)
        acc = (t.astype(np.float64) * t + acc).astype(np.float32)   # fma, exact product
    return acc


def _sphere_d32(x, c, r):
    return (np.sqrt(_f32_sqdist(x, c)).astype(np.float32) - r[None, :]).astype(np.float32)


def _box_d32(x, c, h):
    q = (np.abs((x[:, None, :] - c[None]).astype(np.float32)) - h[None]).astype(np.float32)
    qp = np.maximum(q, np.float32(0))
    out2 = np.zeros(q.shape[:2], np.float32)
    for i in range(q.shape[2]):
        out2 = (qp[..., i].astype(np.float64) * qp[..., i] + out2).astype(np.float32)
    inside = q.max(2)
    return (np.sqrt(out2).astype(np.float32) + np.minimum(inside, np.float32(0))).astype(np.float32)


def _probe_points(rng, c, rad, d, n):
    """Points on, just off, well off and inside member boundaries, plus
    uniform points of the outer box."""
    j = rng.integers(0, len(c), n)
    v = rng.normal(size=(n, d))
    v /= np.linalg.norm(v, axis=1, keepdims=True)
    off = rng.choice([-0.5, -1e-4, 0.0, 1e-6, 1e-4, 1e-2, 0.3, 2.0], n)
    pts = c[j] + v * (rad[j] * (1 + off) + off)[:, None]
    uni = rng.uniform(-np.pi, np.pi, size=(n, d))
    return np.concatenate([pts, uni])


def test_cull_test_is_sound_in_fp32(B):
    """Wherever the FP32 bound says "no member below t" (lb > t), every
    member's FP32 distance exceeds lb, so it exceeds t."""
    shrink = np.float32(1.0 - 2.0 ** -16)
    rng = np.random.default_rng(3)
    for name, s in _sets():
        d = s["d"]
        out = B.wos_debug_clusters(d, s["sph_c"], s["sph_r"], s["box_c"], s["box_h"])
        for kind in ("sph", "box"):
            order, bnd = out[kind]
            if len(order) == 0:
                continue
            if kind == "sph":
                c = np.asarray(s["sph_c"], np.float32)
                r = np.asarray(s["sph_r"], np.float32)
                rad = r.astype(np.float64)
            else:
                c = np.asarray(s["box_c"], np.float32)
                h = np.asarray(s["box_h"], np.float32)
                rad = np.sqrt((h.astype(np.float64) ** 2).sum(1))
            x = _probe_points(rng, c.astype(np.float64), rad, d, 1500).astype(np.float32)
            bc = bnd[:, :-1].astype(np.float32)
            br = bnd[:, -1].astype(np.float32)
            s_ = np.sqrt(_f32_sqdist(x, bc)).astype(np.float32)
            lb = (s_.astype(np.float64) * shrink - br[None, :]).astype(np.float32)   # fma
            dist = _sphere_d32(x, c, r) if kind == "sph" else _box_d32(x, c, h)
            worst = np.inf
            for g in range(len(bnd)):
                m = order[g * CL:(g + 1) * CL]
                m = m[m >= 0]
                gap = dist[:, m].min(1).astype(np.float64) - lb[:, g]
                worst = min(worst, gap.min())
            assert worst > 0, (name, kind, worst)


def _box_lb32(x, lohi, d):
    """The bounding-box test value as the FP32 kernels form it: per axis
    max(lo - x, x - hi, 0), the squares summed by fused multiply-adds, the
    square root, times 1 - 2^-16."""
    lo = lohi[:, :d].astype(np.float32)
    hi = lohi[:, d:].astype(np.float32)
    acc = np.zeros((len(x), len(lo)), np.float32)
    for i in range(d):
        a = (lo[None, :, i] - x[:, None, i]).astype(np.float32)
        b = (x[:, None, i] - hi[None, :, i]).astype(np.float32)
        t = np.maximum(np.maximum(a, b), np.float32(0))
        acc = (t.astype(np.float64) * t + acc).astype(np.float32)   # fma
    return (np.sqrt(acc).astype(np.float32) * np.float32(1.0 - 2.0 ** -16)).astype(np.float32)


def _members(s, kind):
    """FP32 member rows of one kind and the per-axis half extent of each
    member (radius for spheres, half-widths for boxes), in FP64."""
    if kind == "sph":
        c = np.asarray(s["sph_c"], np.float32)
        r = np.asarray(s["sph_r"], np.float32)
        return c, r, np.repeat(r.astype(np.float64)[:, None], c.shape[1], axis=1)
    c = np.asarray(s["box_c"], np.float32)
    h = np.asarray(s["box_h"], np.float32)
    return c, h, h.astype(np.float64)


def test_cluster_boxes_hold_their_members_with_margin(B):
    """Every cluster box contains its members' box enlarged by 2^-16 of that
    box's diagonal on every side (lo and hi as the FP32 device table holds
    them); the boxes are listed in the cluster order of wos_debug_clusters."""
    for name, s in _sets() + _far_tight_sets():
        d = s["d"]
        out = B.wos_debug_clusters(d, s["sph_c"], s["sph_r"], s["box_c"], s["box_h"])
        boxes = B.wos_debug_cluster_boxes(d, s["sph_c"], s["sph_r"], s["box_c"], s["box_h"])
        for kind in ("sph", "box"):
            order, bnd = out[kind]
            lohi = boxes[kind]
            assert lohi.shape == (len(bnd), 2 * d), (name, kind)
            if len(order) == 0:
                continue
            c, _, ext = _members(s, kind)
            assert np.array_equal(lohi.astype(np.float32).astype(np.float64), lohi)
            for g in range(len(bnd)):
                m = order[g * CL:(g + 1) * CL]
                m = m[m >= 0]
                lo = (c[m].astype(np.float64) - ext[m]).min(0)
                hi = (c[m].astype(np.float64) + ext[m]).max(0)
                delta = np.sqrt(((hi - lo) ** 2).sum()) * 2.0 ** -16
                assert np.all(lohi[g, :d] <= lo - delta), (name, kind, g)
                assert np.all(lohi[g, d:] >= hi + delta), (name, kind, g)


def test_box_test_is_sound_in_fp32(B):
    """Wherever the FP32 bounding-box value of a cluster is positive, every
    member's FP32 distance is at least that value, so a pair skipped because
    the value exceeds max(thr, 0) has no member at or below thr.  Probes lie
    on, just off and inside members, just past members' extreme points along
    the axes (where a member touches its cluster's box), just outside the
    faces and corners of the cluster boxes, and uniformly in the outer box."""
    rng = np.random.default_rng(12)
    for name, s in _sets() + _far_tight_sets():
        d = s["d"]
        out = B.wos_debug_clusters(d, s["sph_c"], s["sph_r"], s["box_c"], s["box_h"])
        boxes = B.wos_debug_cluster_boxes(d, s["sph_c"], s["sph_r"], s["box_c"], s["box_h"])
        for kind in ("sph", "box"):
            order, _ = out[kind]
            lohi = boxes[kind]
            if len(order) == 0:
                continue
            c, r_or_h, ext = _members(s, kind)
            rad = np.sqrt((ext ** 2).sum(1)) if kind == "box" else ext[:, 0]
            x = _probe_points(rng, c.astype(np.float64), rad, d, 800)
            g = rng.integers(0, len(lohi), 800)
            # just outside a face or a corner of a cluster box
            side = rng.integers(0, 2, size=(800, d))
            corner = np.where(side, lohi[g, d:], lohi[g, :d])
            face = rng.uniform(lohi[g, :d], lohi[g, d:])
            ax = rng.integers(0, d, 800)
            face[np.arange(800), ax] = corner[np.arange(800), ax]
            off = rng.choice([0.0, 1e-7, 1e-5, 1e-3], size=(800, 1))
            push = np.where(side, 1.0, -1.0) * off
            # just past a member's extreme point along an axis, where its
            # surface touches its cluster's box face: the tightest case
            j = rng.integers(0, len(c), 800)
            ax = rng.integers(0, d, 800)
            sg = rng.choice([-1.0, 1.0], 800)
            tip = c[j].astype(np.float64)
            tip[np.arange(800), ax] += sg * (ext[j, ax] + rng.choice([0.0, 1e-7, 1e-5, 1e-3], 800))
            x = np.concatenate([x, corner + push, face + push, tip]).astype(np.float32)
            dist = _sphere_d32(x, c, r_or_h) if kind == "sph" else _box_d32(x, c, r_or_h)
            lb = _box_lb32(x, lohi, d)
            worst = np.inf
            for k in range(len(lohi)):
                m = order[k * CL:(k + 1) * CL]
                m = m[m >= 0]
                pos = lb[:, k] > 0
                if pos.any():
                    gap = dist[pos][:, m].min(1).astype(np.float64) - lb[pos, k]
                    worst = min(worst, gap.min())
            assert worst >= 0, (name, kind, worst)


def test_box_test_tightens_the_sphere_bound(B):
    """On the 7-D segment workload the walker's threshold is mostly the
    outer-box distance; of the (query, cluster) pairs whose bounding sphere
    comes within that threshold, the bounding box rules out most."""
    s = S.scene_c3(n_walks=16)
    d = s["d"]
    out = B.wos_debug_clusters(d, s["sph_c"], s["sph_r"])
    lohi = B.wos_debug_cluster_boxes(d, s["sph_c"], s["sph_r"])["sph"]
    _, bnd = out["sph"]
    x = np.asarray(s["queries"], np.float32)
    thr = np.minimum(np.pi - np.abs(x.astype(np.float64)).max(1),
                     np.linalg.norm(x - s["goal_c"], axis=1) - s["goal_r"])
    sphere_lb = np.linalg.norm(x[:, None].astype(np.float64) - bnd[None, :, :-1], axis=2) - bnd[None, :, -1]
    kept = sphere_lb <= thr[:, None]
    box_out = _box_lb32(x, lohi, d) > thr[:, None]
    assert kept.sum() > 0
    assert (kept & box_out).sum() > 0.5 * kept.sum()


def test_cull_test_is_sound_in_fp64(B):
    shrink = 1.0 - 2.0 ** -45
    rng = np.random.default_rng(4)
    for name, s in _sets():
        d = s["d"]
        out = B.wos_debug_clusters(d, s["sph_c"], s["sph_r"], s["box_c"], s["box_h"], fp64=True)
        order, bnd = out["sph"]
        if len(order) == 0:
            continue
        c, r = np.asarray(s["sph_c"]), np.asarray(s["sph_r"])
        x = _probe_points(rng, c, r, d, 1000)
        dist = np.sqrt(((x[:, None] - c[None]) ** 2).sum(2)) - r[None]
        lb = np.sqrt(((x[:, None] - bnd[None, :, :-1]) ** 2).sum(2)) * shrink - bnd[None, :, -1]
        for g in range(len(bnd)):
            m = order[g * CL:(g + 1) * CL]
            m = m[m >= 0]
            assert np.all(dist[:, m].min(1) > lb[:, g]), (name, g)


def test_bounds_cull_far_points(B):
    """The bounds are not vacuous: from a point far outside an obstacle set
    most clusters are provably farther than the nearest obstacle."""
    s = S.scene_c4_env(5, n_walks=16, q_cap=4)
    d = s["d"]
    out = B.wos_debug_clusters(d, s["sph_c"], s["sph_r"])
    order, bnd = out["sph"]
    c, r = np.asarray(s["sph_c"]), np.asarray(s["sph_r"])
    x = np.asarray(s["queries"][:4])
    R = (np.sqrt(((x[:, None] - c[None]) ** 2).sum(2)) - r[None]).min(1)
    lb = np.sqrt(((x[:, None] - bnd[None, :, :-1]) ** 2).sum(2)) - bnd[None, :, -1]
    assert (lb > R[:, None]).mean() > 0.3


def test_debug_clusters_rejects_bad_input(B):
    import ctypes as C
    n = (C.c_int64 * 2)()
    assert B.lib.wos_debug_clusters(9, None, None, 0, n, None, None, None, None) == B.WOS_EDIM
    assert B.lib.wos_debug_clusters(3, None, None, 0, None, None, None, None, None) == B.WOS_EINVAL
    with pytest.raises(B.WosError):
        B.wos_debug_clusters(3, np.zeros((70, 3)), -np.ones(70))


def test_debug_cluster_boxes_rejects_bad_input(B):
    import ctypes as C
    n = (C.c_int64 * 2)()
    assert B.lib.wos_debug_cluster_boxes(1, None, None, n, None, None) == B.WOS_EDIM
    assert B.lib.wos_debug_cluster_boxes(3, None, None, None, None, None) == B.WOS_EINVAL
    with pytest.raises(B.WosError):
        B.wos_debug_cluster_boxes(3, np.zeros((70, 3)), -np.ones(70))
    # no obstacles, or fewer than 64: no clusters, no boxes
    out = B.wos_debug_cluster_boxes(3, np.zeros((10, 3)), np.ones(10))
    assert out["sph"].shape == (0, 6) and out["box"].shape == (0, 6)


def _mfma_features(x, thr, bc, br, d):
    """Walker features (FP32, as the kernel forms them) and cluster features
    (FP64 rounded once to FP32, as the host forms them) of the matrix-core
    cluster test, m = 2^-12."""
    m = np.float32(2.0 ** -12)
    n = len(x)
    a = np.zeros((n, 12), np.float32)
    a[:, :d] = x
    xx = np.zeros(n, np.float32)
    for i in range(d):
        xx = (x[:, i].astype(np.float64) * x[:, i] + xx).astype(np.float32)       # fma
    mt2 = ((m * thr).astype(np.float32) * thr).astype(np.float32)
    a[:, 8] = (xx.astype(np.float64) * np.float32(1 - m) - mt2).astype(np.float32)  # fma
    a[:, 9] = 1.0
    a[:, 10] = (thr * thr).astype(np.float32)
    a[:, 11] = thr
    md = 2.0 ** -12
    b = np.zeros((len(bc), 12), np.float32)
    cc = (bc.astype(np.float64) ** 2).sum(1)
    rho = br.astype(np.float64)
    b[:, :d] = (-2.0 * bc.astype(np.float64)).astype(np.float32)
    b[:, 8] = 1.0
    b[:, 9] = (cc * (1 - md) - rho * rho * (1 + md)).astype(np.float32)
    b[:, 10] = -1.0
    b[:, 11] = (-2.0 * rho).astype(np.float32)
    return a, b


def _dot32(a, b, order):
    """FP32 dot products of every row of a with every row of b, three ways a
    4-deep matrix step may round: a chain of fused multiply-adds in feature
    order or reversed, or rounded products summed in pairs per step of 4."""
    A = a.astype(np.float64)[:, None, :]
    Bm = b.astype(np.float64)[None, :, :]
    acc = np.zeros((a.shape[0], b.shape[0]), np.float32)
    if order == "fma":
        for k in range(12):
            acc = (A[..., k] * Bm[..., k] + acc).astype(np.float32)
    elif order == "reverse":
        for k in reversed(range(12)):
            acc = (A[..., k] * Bm[..., k] + acc).astype(np.float32)
    else:
        for s in range(3):
            p = [(A[..., 4 * s + k] * Bm[..., 4 * s + k]).astype(np.float32) for k in range(4)]
            s01 = (p[0] + p[1]).astype(np.float32)
            s23 = (p[2] + p[3]).astype(np.float32)
            acc = (acc + (s01 + s23).astype(np.float32)).astype(np.float32)
    return acc


def _far_tight_sets():
    """Point obstacles (radius 0) packed near (7, 7, ...): large |x|^2 and
    |C|^2 against small cluster radii, where the FP32 rounding of the expanded
    dot product is largest relative to the cluster bound's own slack."""
    out = []
    for d, seed in ((3, 21), (7, 22)):
        rng = np.random.default_rng(seed)
        c = 7.0 + rng.normal(scale=0.15, size=(256, d))
        s = S._empty(d)
        s.update(d=d, sph_c=c, sph_r=np.zeros(256))
        out.append((f"far_tight_d{d}", s))
    return out


@pytest.mark.parametrize("order", ["fma", "reverse", "pairs"])
def test_matrix_core_cull_test_is_sound_in_fp32(B, order):
    """Wherever the matrix-core test skips a cluster for a walker (the FP32
    feature dot product, in any of three rounding orders, has its sign bit
    clear: +0 included, since the margin dwarfs the rounding), every member's
    FP32 distance exceeds the walker's threshold: thresholds are put at, just
    below and just above the exact bound, the hardest cases."""
    rng = np.random.default_rng(11)
    for name, s in _sets() + _far_tight_sets():
        d = s["d"]
        out = B.wos_debug_clusters(d, s["sph_c"], s["sph_r"], s["box_c"], s["box_h"])
        for kind in ("sph", "box"):
            order_, bnd = out[kind]
            if len(order_) == 0:
                continue
            if kind == "sph":
                c = np.asarray(s["sph_c"], np.float32)
                r = np.asarray(s["sph_r"], np.float32)
                rad = r.astype(np.float64)
            else:
                c = np.asarray(s["box_c"], np.float32)
                h = np.asarray(s["box_h"], np.float32)
                rad = np.sqrt((h.astype(np.float64) ** 2).sum(1))
            x = _probe_points(rng, c.astype(np.float64), rad, d, 400).astype(np.float32)
            bc = bnd[:, :-1].astype(np.float32)
            br = bnd[:, -1].astype(np.float32)
            exact_lb = np.linalg.norm(x.astype(np.float64)[:, None] - bc.astype(np.float64)[None], axis=2) \
                - br.astype(np.float64)[None]
            dist = _sphere_d32(x, c, r) if kind == "sph" else _box_d32(x, c, h)
            member_min = np.stack([dist[:, order_[g * CL:(g + 1) * CL][order_[g * CL:(g + 1) * CL] >= 0]].min(1)
                                   for g in range(len(bnd))], axis=1)
            checked = 0
            for rel in (-1e-3, -1e-5, 0.0, 1e-5, 1e-3):
                g = rng.integers(0, len(bnd), len(x))
                thr = np.maximum(exact_lb[np.arange(len(x)), g] * (1 + rel), 1e-6).astype(np.float32)
                a, b = _mfma_features(x, thr, bc, br, d)
                D = _dot32(a, b, order)
                skip = ~np.signbit(D)
                bad = skip & ~(member_min > thr[:, None])
                assert not bad.any(), (name, kind, rel, np.argwhere(bad)[:3])
                checked += skip.sum()
            assert checked > 0


def test_step_bound_holds_in_fp32():
    """The walkers' step-to-step bound: R at a step is at most twice R at
    the step before (a minimum of 1-Lipschitz distances; the walker moves
    R), and the FP32 walk stays within the kernels' margins, 2 R (1 + 2^-10)
    + 2^-14 (1 + size of the geometry).  Walks emulated in FP32 (positions
    updated by a rounded multiply-add, distances as the kernels form them) in
    dense 3- and 4-D sphere scenes and a 7-D one, where the ratio comes
    closest to 2 (steps towards a near obstacle)."""
    rng = np.random.default_rng(21)
    worst = -np.inf
    for e in (105, 1, 61, 7):
        s = S.scene_c4_env(e, n_walks=16, q_cap=64)
        d = s["d"]
        c = np.asarray(s["sph_c"], np.float32)
        r = np.asarray(s["sph_r"], np.float32)
        lo, hi = np.float32(-np.pi), np.float32(np.pi)
        scale = max(np.abs(c).max() + r.max(), np.pi, np.abs(s["goal_c"]).max() + s["goal_r"])
        x = np.asarray(s["queries"], np.float32)[:64].copy()
        Rp = None
        for _ in range(60):
            dout = np.minimum(x - lo, hi - x).min(1).astype(np.float32)
            gc = np.asarray(s["goal_c"], np.float32)
            dg = (np.sqrt(_f32_sqdist(x, gc[None])[:, 0]).astype(np.float32) - np.float32(s["goal_r"])).astype(np.float32)
            R = np.minimum(np.minimum(dout, dg), _sphere_d32(x, c, r).min(1)).astype(np.float32)
            if Rp is not None:
                ok = Rp > 0
                bound = (Rp[ok].astype(np.float64) * 2.001953125 + 2.0 ** -14 * (1.0 + scale))
                assert np.all(R[ok] <= bound), (e, np.max(R[ok] - bound))
                worst = max(worst, float(np.max(R[ok] / np.maximum(Rp[ok], 1e-30))))
            v = rng.normal(size=x.shape).astype(np.float32)
            v = (v / np.sqrt((v.astype(np.float64) ** 2).sum(1, keepdims=True))).astype(np.float32)
            Rc = np.maximum(R, np.float32(0))
            x = (Rc[:, None].astype(np.float64) * v + x).astype(np.float32)   # fma
            Rp = Rc
    assert worst > 1.5   # the bound is approached
