"""Pins of the CPU oracle against what the paper and the mathematics fix.

Each test checks the oracle against something other than itself: printed or
hand-derived values (tests/golden), closed forms, invariants, a library
routine (scipy), or the pure-Python brute force in tests/brute.py, which
restates every stage in a different form.
"""
import itertools
import os

import numpy as np
import pytest
import scipy.ndimage
import scipy.sparse
import scipy.sparse.csgraph

import brute
import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _to_lists(f):
    return [[tuple(int(c) for c in f[y, x]) for x in range(f.shape[1])] for y in range(f.shape[0])]


# ---------------------------------------------------------------- O1 luma
def test_luma_all_colours(oracle_mod):
    """All 2^24 colours: grey maps to itself (weights sum to 256) and the
    value stays within 1.5 of BT.601 luma 0.299R + 0.587G + 0.114B."""
    v = np.arange(1 << 24, dtype=np.uint32)
    rgb = np.stack([(v >> 16) & 255, (v >> 8) & 255, v & 255], -1).astype(np.uint8)
    Y = oracle_mod.luma(rgb).astype(np.float64)
    ref = rgb[:, 0] * 0.299 + rgb[:, 1] * 0.587 + rgb[:, 2] * 0.114
    assert np.abs(Y - ref).max() <= 1.5
    assert abs(np.mean(Y - ref)) < 0.5
    grey = np.repeat(np.arange(256, dtype=np.uint8)[:, None], 3, 1)
    assert np.array_equal(oracle_mod.luma(grey), np.arange(256, dtype=np.uint8))
    # brute force on a random sample
    rng = np.random.default_rng(11)
    idx = rng.integers(0, 1 << 24, 2000)
    assert all(int(Y[i]) == brute.luma(*map(int, rgb[i])) for i in idx)


# ----------------------------------------------------------- O9 tables
def _golden_tables():
    t = {}
    for line in open(os.path.join(GOLDEN, "cbf_tables.txt")):
        if line.startswith("#") or not line.strip():
            continue
        name, *vals = line.split()
        t[name] = [int(v) for v in vals]
    return t


def test_weight_tables_normative(oracle_mod):
    ws, wr = oracle_mod.weight_tables()
    g = _golden_tables()
    assert list(ws) == g["ws"]
    assert list(wr[:43]) == g["wr"]
    assert not wr[43:].any()
    bws, bwr = brute.weight_tables(3)
    assert list(ws) == bws and list(wr) == bwr


def test_weight_table_margins():
    """Every table entry is far from a half-integer, so any correctly rounded
    double exp() gives the same integers."""
    k = np.arange(19)
    d = np.arange(256)
    a = 255 * np.exp(-k / 4.5)
    b = 255 * np.exp(-(d * d) / 288.0)
    for v in (a, b):
        frac = v - np.floor(v)
        assert np.min(np.abs(frac - 0.5)) > 9e-4


# ------------------------------------------------------------- O10 LUT
def test_disparity_lut_golden(oracle_mod):
    rows = [list(map(int, l.split())) for l in open(os.path.join(GOLDEN, "disparity_lut.txt"))
            if l.strip() and not l.startswith("#")]
    assert len(rows) >= 10
    for B, T, D, P, oL, oR in rows:
        p, l, r = oracle_mod.disparity_lut(B, T)
        assert (p[D], l[D], r[D]) == (P, oL, oR), (B, T, D)
        assert brute.parallax(B, T, D) == (P, oL, oR)


@pytest.mark.parametrize("B", [0, 1, 7, 12, 38, 77, 154, 255])
def test_disparity_lut_properties(oracle_mod, B):
    """Against the Fig. 3 formulas: each view moves by about half the base
    times D/255 (crossed) or (1 - D/255) (uncrossed), in opposite directions;
    the total is the nearest integer to the real parallax; P is monotone."""
    for T in (150, -1, 0, 254):
        P, oL, oR = oracle_mod.disparity_lut(B, T)
        D = np.arange(256)
        crossed = D > T
        real = np.where(crossed, B * D / 255.0, -B * (255 - D) / 255.0)
        assert np.all(np.abs(P - real) <= 0.5 + 1e-12)
        assert np.array_equal(oL - oR, P)
        # each view is within 3/4 px of half the real parallax: half of the
        # rounding of P plus the odd pixel given to the left view
        assert np.all(np.abs(oL - real / 2) <= 0.75 + 1e-12)
        assert np.all(np.abs(oR + real / 2) <= 0.75 + 1e-12)
        assert np.all((oL + oR == 0) | (oL + oR == np.sign(P)))
        assert np.all(np.sign(oL[crossed]) >= 0) and np.all(np.sign(oL[~crossed]) <= 0)
        assert np.all(np.diff(P) >= 0)
        assert P.min() >= -B and P.max() <= B


# ---------------------------------------------------------------- O2 K
@pytest.mark.parametrize("w,h,K,grid", [
    (640, 360, 8, (80, 45)), (1920, 1080, 8, (240, 135)), (3840, 2160, 16, (240, 135)),
    (7680, 4320, 32, (240, 135)), (1280, 720, 8, (160, 90)), (2560, 1440, 16, (160, 90)),
    (1, 1, 8, (1, 1))])
def test_auto_block(oracle_mod, w, h, K, grid):
    assert oracle_mod.auto_block(w, h) == K
    assert (-(-w // K), -(-h // K)) == grid


# ----------------------------------------------------- O5-O6 components
def _links_from_stats(stats, tau):
    gh, gw = stats.shape
    e = (stats >> 24) & 1
    mu = np.stack([(stats >> (8 * c)) & 255 for c in range(3)], -1).astype(np.int64)
    rows, cols = [], []
    for by in range(gh):
        for bx in range(gw):
            b = by * gw + bx
            if e[by, bx]:
                continue
            if bx + 1 < gw and not e[by, bx + 1] and np.abs(mu[by, bx] - mu[by, bx + 1]).sum() <= tau:
                rows.append(b); cols.append(b + 1)
            if by + 1 < gh and not e[by + 1, bx] and np.abs(mu[by, bx] - mu[by + 1, bx]).sum() <= tau:
                rows.append(b); cols.append(b + gw)
    n = gh * gw
    return scipy.sparse.coo_matrix((np.ones(len(rows)), (rows, cols)), shape=(n, n))


def _scipy_labels(stats, tau):
    n = stats.size
    _, comp = scipy.sparse.csgraph.connected_components(_links_from_stats(stats, tau), directed=False)
    mins = np.full(comp.max() + 1, n)
    np.minimum.at(mins, comp, np.arange(n))
    return mins[comp].reshape(stats.shape)


@pytest.mark.parametrize("seed,w,h,K", [(1, 640, 360, 8), (2, 320, 240, 4), (3, 333, 191, 8),
                                        (4, 1920, 1080, 8)])
def test_labels_match_scipy(oracle_mod, seed, w, h, K):
    f = synth.gen_frame(seed, w, h, 30, 4.0)
    o = oracle_mod.synthesize(f, 12, K=K)
    assert np.array_equal(o.labels, _scipy_labels(o.stats, 24))
    # edge blocks are singletons
    e = (o.stats >> 24).astype(bool)
    idx = np.arange(o.labels.size).reshape(o.labels.shape)
    assert np.array_equal(o.labels[e], idx[e])


def _serpentine_frame(gw, gh, K):
    """Path blocks form one snake; wall blocks differ by 30 in red (mean L1
    distance 30 > tau, luma step 9 <= g): no edges, no links across."""
    f = np.zeros((gh * K, gw * K, 3), np.uint8)
    f[:] = (130, 100, 100)
    for by in range(gh):
        if by % 2 == 0:
            f[by * K:(by + 1) * K, :, :] = (100, 100, 100)
        else:
            bx = gw - 1 if (by // 2) % 2 == 0 else 0
            f[by * K:(by + 1) * K, bx * K:(bx + 1) * K, :] = (100, 100, 100)
    return f


def test_labels_serpentine(oracle_mod):
    f = _serpentine_frame(40, 31, 4)
    o = oracle_mod.synthesize(f, 12, K=4)
    assert not (o.stats >> 24).any()
    assert np.array_equal(o.labels, _scipy_labels(o.stats, 24))
    snake = np.all(f[::4, ::4] == (100, 100, 100), -1)
    assert np.all(o.labels[snake] == 0)


# ------------------------------------------------------- O7-O8 depth
def test_uniform_frame_is_ramp(oracle_mod):
    """One background region: every pixel takes the ramp of its block row."""
    f = np.full((90, 160, 3), 77, np.uint8)
    o = oracle_mod.synthesize(f, 12, K=8)
    gh = 90 // 8 + 1
    ramp = [int(np.floor(255 * r / (gh - 1) + 0.5)) for r in range(gh)]
    rows = np.arange(90) // 8
    assert np.array_equal(o.D0, np.repeat(np.array(ramp, np.uint8)[rows][:, None], 160, 1))
    assert (o.labels == 0).all()


def test_all_edge_frame(oracle_mod):
    """Every block has an edge: pixel depth falls back to the block-row ramp."""
    f = np.zeros((32, 48, 3), np.uint8)
    f[:, ::2] = 255
    o = oracle_mod.synthesize(f, 12, K=8)
    assert ((o.stats >> 24) == 1).all()
    ramp = np.array([0, 85, 170, 255], np.uint8)
    assert np.array_equal(o.D0, np.repeat(ramp[np.arange(32) // 8][:, None], 48, 1))


# ------------------------------------------------------------- O9 CBF
def test_cbf_radius0_is_identity(oracle_mod):
    f = synth.gen_frame(5, 96, 64, 8, 4.0)
    o = oracle_mod.synthesize(f, 12, K=8, r=0)
    assert np.array_equal(o.Df, o.D0)


def test_cbf_constant_depth(oracle_mod):
    f = synth.gen_frame(6, 96, 64, 8, 4.0)
    for c in (0, 1, 150, 151, 254, 255):
        o = oracle_mod.synthesize(f, 12, depth=np.full((64, 96), c, np.uint8))
        assert (o.Df == c).all()


@pytest.mark.parametrize("r", [1, 2, 3])
def test_cbf_constant_luma_is_gaussian(oracle_mod, r):
    """Constant guide: range weight is 255 everywhere and the filter is a
    normalised integer Gaussian, clipped at the borders; checked with
    scipy.ndimage.correlate in float64 (exact on these integers)."""
    rng = np.random.default_rng(r)
    h, w = 37, 53
    D0 = rng.integers(0, 256, (h, w)).astype(np.uint8)
    f = np.full((h, w, 3), 120, np.uint8)
    ws = [int(np.floor(255 * np.exp(-k / 4.5) + 0.5)) for k in range(19)]
    ker = np.array([[ws[dx * dx + dy * dy] for dx in range(-r, r + 1)] for dy in range(-r, r + 1)], np.float64)
    num = scipy.ndimage.correlate(D0.astype(np.float64), ker, mode="constant", cval=0.0) * 255
    den = scipy.ndimage.correlate(np.ones((h, w)), ker, mode="constant", cval=0.0) * 255
    num, den = num.astype(np.int64), den.astype(np.int64)
    expect = (num + den // 2) // den
    o = oracle_mod.synthesize(f, 12, depth=D0, r=r)
    assert np.array_equal(o.Df.astype(np.int64), expect)


# ---------------------------------------------------------- invariants
@pytest.mark.parametrize("seed", [1, 2, 3])
def test_I1_zero_base_identity(oracle_mod, seed):
    """B = 0: both views and the anaglyph equal the source frame."""
    f = synth.gen_frame(seed, 200, 120, 12, 4.0)
    o = oracle_mod.synthesize(f, 0)
    assert np.array_equal(o.L, f) and np.array_equal(o.R, f) and np.array_equal(o.A, f)


def test_I1_linear_mode_zero_depth(oracle_mod):
    f = synth.gen_frame(9, 150, 70, 12, 4.0)
    o = oracle_mod.synthesize(f, 12, T=-1, depth=np.zeros((70, 150), np.uint8))
    assert np.array_equal(o.L, f) and np.array_equal(o.R, f) and np.array_equal(o.A, f)


@pytest.mark.parametrize("D", [0, 100, 150, 151, 200, 255])
@pytest.mark.parametrize("B", [12, 38, 77])
def test_I3_constant_depth_translation(oracle_mod, D, B):
    """Constant depth: each view is the source shifted by its offset; the
    uncovered border strip repeats the nearest warped pixel.  The Fig. 3
    gather gives the same interior."""
    h, w = 9, 160
    f = synth.gen_frame(D + B, w, h, 5, 4.0)
    o = oracle_mod.synthesize(f, B, depth=np.full((h, w), D, np.uint8))
    _, oL, oR = oracle_mod.disparity_lut(B)
    for V, off in ((o.L, oL[D]), (o.R, oR[D])):
        xs = np.arange(w)
        src = np.clip(xs - off, 0, w - 1)
        assert np.array_equal(V, f[:, src])


def test_I2_z_order(oracle_mod):
    """At a collision the nearer (larger depth) source wins."""
    h, w = 3, 64
    f = synth.gen_frame(4, w, h, 4, 4.0)
    dep = np.zeros((h, w), np.uint8)
    dep[:, 20:28] = 255
    o = oracle_mod.synthesize(f, 12, depth=dep, r=0)
    _, oL, _ = oracle_mod.disparity_lut(12)
    for x in range(20, 28):
        xd = x + oL[255]
        # the background source xd - oL[0] lands on the same destination
        assert 0 <= xd - oL[0] < w and dep[0, xd - oL[0]] == 0
        assert (o.warpL[:, xd] == x).all()


def _check_fill(o, w):
    for wp, sp in ((o.warpL, o.srcL), (o.warpR, o.srcR)):
        assert (sp >= 0).all() and (sp < w).all()
        for y in range(wp.shape[0]):
            valid = set(int(v) for v in wp[y] if v >= 0)
            if valid:
                assert set(int(v) for v in sp[y]) <= valid
            else:
                assert np.array_equal(sp[y], np.arange(w))
            nh = wp[y] >= 0
            assert np.array_equal(sp[y][nh], wp[y][nh])


@pytest.mark.parametrize("seed", [1, 7])
def test_I4_I6_fill(oracle_mod, seed):
    """No holes remain; each filled colour copies a warped pixel of its row
    (or the source pixel in an empty row); non-holes are untouched."""
    f = synth.gen_frame(seed, 320, 90, 20, 4.0)
    o = oracle_mod.synthesize(f, 38, K=8)
    _check_fill(o, 320)
    # at least some holes were actually filled
    assert (o.warpL < 0).any() and (o.warpR < 0).any()


def test_I6_no_hole_identity(oracle_mod):
    h, w = 4, 40
    f = synth.gen_frame(2, w, h, 3, 4.0)
    o = oracle_mod.synthesize(f, 0, depth=np.full((h, w), 77, np.uint8))
    assert (o.warpL >= 0).all()
    assert np.array_equal(o.srcL, o.warpL)


def test_empty_row_copies_source(oracle_mod):
    """Every source leaves the row: the row falls back to the source pixels."""
    h, w = 2, 6
    f = synth.gen_frame(3, w, h, 2, 4.0)
    o = oracle_mod.synthesize(f, 255, depth=np.full((h, w), 255, np.uint8))
    assert (o.warpL < 0).all() and (o.warpR < 0).all()
    assert np.array_equal(o.L, f) and np.array_equal(o.R, f)


def test_I5_mirror(oracle_mod):
    """With every parallax even, mirroring the input swaps the views (mirrored)."""
    B = 12
    P, _, _ = oracle_mod.disparity_lut(B)
    even = [d for d in range(256) if P[d] % 2 == 0]
    rng = np.random.default_rng(3)
    h, w = 6, 48
    dep = rng.choice(even, (h, w)).astype(np.uint8)
    f = synth.gen_frame(8, w, h, 3, 4.0)
    o = oracle_mod.synthesize(f, B, depth=dep, r=0)
    m = oracle_mod.synthesize(f[:, ::-1].copy(), B, depth=dep[:, ::-1].copy(), r=0)
    assert np.array_equal(m.L, o.R[:, ::-1]) and np.array_equal(m.R, o.L[:, ::-1])


# ---------------------------------------------------- worked examples
def _worked_rows():
    out = []
    for line in open(os.path.join(GOLDEN, "worked_rows.txt")):
        if line.startswith("#") or not line.strip():
            continue
        name, dep, L, R = [s.strip() for s in line.split("|")]
        out.append((name, [int(v) for v in dep.split()], [int(v) for v in L.split()],
                    [int(v) for v in R.split()]))
    return out


@pytest.mark.parametrize("case", _worked_rows(), ids=lambda c: c[0])
def test_worked_examples(oracle_mod, case):
    name, dep, Ls, Rs = case
    w = len(dep)
    f = np.zeros((1, w, 3), np.uint8)
    f[0, :, 0] = np.arange(w) * 10
    f[0, :, 1] = 255 - np.arange(w) * 10
    f[0, :, 2] = 7
    o = oracle_mod.synthesize(f, 12, T=150, depth=np.array([dep], np.uint8), r=0)
    assert list(o.srcL[0]) == Ls
    assert list(o.srcR[0]) == Rs
    assert np.array_equal(o.L[0], f[0, Ls]) and np.array_equal(o.R[0], f[0, Rs])
    b = brute.pipeline(_to_lists(f), 12, 150, K=8, r=0, depth=[dep])
    assert b["srcL"][0] == Ls and b["srcR"][0] == Rs


# ------------------------------------------------------- brute force
def test_brute_exhaustive_rows(oracle_mod):
    """Every 1x4 row over depths {0,150,151,255} and B in 0..8."""
    f = np.zeros((1, 4, 3), np.uint8)
    f[0, :, 0] = [10, 20, 30, 40]
    for B in range(9):
        for dep in itertools.product((0, 150, 151, 255), repeat=4):
            o = oracle_mod.synthesize(f, B, depth=np.array([dep], np.uint8), r=0)
            b = brute.pipeline(_to_lists(f), B, 150, K=8, r=0, depth=[list(dep)])
            assert list(o.srcL[0]) == b["srcL"][0] and list(o.srcR[0]) == b["srcR"][0], (B, dep)
            assert list(o.warpL[0]) == b["warpL"][0] and list(o.warpR[0]) == b["warpR"][0]


STAGES = ["Y", "stats", "labels", "dblk", "D0", "Df", "warpL", "warpR", "srcL", "srcR", "L", "R", "A"]


@pytest.mark.parametrize("trial", range(40))
def test_brute_random_small(oracle_mod, trial):
    rng = np.random.default_rng(1000 + trial)
    w, h = int(rng.integers(1, 17)), int(rng.integers(1, 13))
    K = int(rng.choice([1, 2, 3, 4, 8]))
    B = int(rng.integers(0, 24))
    T = int(rng.choice([-1, 0, 100, 150, 200, 255]))
    r = int(rng.integers(0, 4))
    g = int(rng.choice([0, 8, 24, 60]))
    tau = int(rng.choice([0, 12, 24, 80]))
    if trial % 3 == 0:
        f = rng.integers(0, 256, (h, w, 3)).astype(np.uint8)
    else:
        f = synth.gen_frame(trial, w, h, 4, 4.0)
    o = oracle_mod.synthesize(f, B, T, K, g, tau, r)
    b = brute.pipeline(_to_lists(f), B, T, K, g, tau, r)
    for k in STAGES:
        assert np.array_equal(getattr(o, k).astype(np.int64), np.array(b[k], np.int64)), k


@pytest.mark.parametrize("seed", [1, 2])
def test_brute_8x8_and_24x16(oracle_mod, seed):
    for (w, h, K) in ((8, 8, 2), (8, 8, 4), (24, 16, 4)):
        f = synth.gen_frame(seed, w, h, 3, 4.0)
        o = oracle_mod.synthesize(f, 6, K=K)
        b = brute.pipeline(_to_lists(f), 6, K=K)
        for k in STAGES:
            assert np.array_equal(getattr(o, k).astype(np.int64), np.array(b[k], np.int64)), k


def test_oracle_rejects_bad_args(oracle_mod):
    f = np.zeros((4, 4, 3), np.uint8)
    for kw in ({"B": -1}, {"B": 256}, {"T": -2}, {"r": 4}):
        args = {"B": 12}
        args.update(kw)
        with pytest.raises(ValueError):
            oracle_mod.synthesize(f, **args)


# ------------------------------------------------------------ HSBS output
@pytest.mark.parametrize("w,h,seed", [(1, 1, 0), (2, 3, 1), (7, 2, 2), (8, 5, 3), (33, 4, 4), (64, 2, 5)])
def test_hsbs_brute_force(oracle_mod, w, h, seed):
    rng = np.random.default_rng(seed)
    L = rng.integers(0, 256, (h, w, 3), dtype=np.uint8)
    R = rng.integers(0, 256, (h, w, 3), dtype=np.uint8)
    got = oracle_mod.hsbs(L, R)
    want = np.array(brute.hsbs(L.tolist(), R.tolist()), dtype=np.uint8).reshape(h, w, 3)
    assert np.array_equal(got, want)


def test_hsbs_closed_forms(oracle_mod):
    # a constant pair stays constant; equal views give equal halves; odd
    # widths copy the right view's last column; 255/0 neighbours round up
    c = np.full((3, 10, 3), 77, np.uint8)
    assert np.array_equal(oracle_mod.hsbs(c, c), c)
    rng = np.random.default_rng(9)
    v = rng.integers(0, 256, (4, 12, 3), dtype=np.uint8)
    hs = oracle_mod.hsbs(v, v)
    assert np.array_equal(hs[:, :6], hs[:, 6:])
    odd = rng.integers(0, 256, (2, 9, 3), dtype=np.uint8)
    assert np.array_equal(oracle_mod.hsbs(odd, odd)[:, 8], odd[:, 8])
    pair = np.zeros((1, 2, 3), np.uint8)
    pair[0, 1] = 255
    assert oracle_mod.hsbs(pair, pair)[0, 0].tolist() == [128, 128, 128]
    assert oracle_mod.hsbs(pair, pair)[0, 1].tolist() == [128, 128, 128]


# ------------------------------------------------ Fig. 3 gather warp
def _gather_rows():
    out = []
    for line in open(os.path.join(GOLDEN, "gather_rows.txt")):
        if line.startswith("#") or not line.strip():
            continue
        name, dep, L, R = [s.strip() for s in line.split("|")]
        out.append((name, [int(v) for v in dep.split()], [int(v) for v in L.split()],
                    [int(v) for v in R.split()]))
    return out


@pytest.mark.parametrize("case", _gather_rows(), ids=lambda c: c[0])
def test_gather_worked_rows(oracle_mod, case):
    name, dep, Ls, Rs = case
    w = len(dep)
    f = np.zeros((1, w, 3), np.uint8)
    f[0, :, 0] = np.arange(w) * 10
    f[0, :, 1] = 255 - np.arange(w) * 10
    f[0, :, 2] = 7
    L, R, A = oracle_mod.synthesize_gather(f, 12, T=150, depth=np.array([dep], np.uint8), r=0)
    assert np.array_equal(L[0], f[0, Ls]) and np.array_equal(R[0], f[0, Rs])
    assert np.array_equal(A[0, :, 0], L[0, :, 0]) and np.array_equal(A[0, :, 1:], R[0, :, 1:])


@pytest.mark.parametrize("seed", range(6))
def test_gather_brute_force(oracle_mod, seed):
    rng = np.random.default_rng(300 + seed)
    h, w = int(rng.integers(1, 6)), int(rng.integers(1, 40))
    f = rng.integers(0, 256, (h, w, 3), dtype=np.uint8)
    Df = rng.choice(np.array([0, 90, 150, 151, 200, 255], np.uint8), (h, w))
    B, T = int(rng.integers(0, 60)), int(rng.choice([-1, 150, 100]))
    got = oracle_mod.gather(f, Df, B, T)
    want = brute.gather(f.tolist(), Df.tolist(), B, T)
    for g_, w_ in zip(got, want):
        assert np.array_equal(g_, np.array(w_, np.uint8).reshape(h, w, 3))


def test_gather_invariants(oracle_mod):
    rng = np.random.default_rng(77)
    f = rng.integers(0, 256, (6, 50, 3), dtype=np.uint8)
    # B = 0: every view is the input
    L, R, A = oracle_mod.synthesize_gather(f, 0)
    assert np.array_equal(L, f) and np.array_equal(R, f) and np.array_equal(A, f)
    # constant depth: same interior as the z-buffered forward warp (a pure
    # translation), while the border strip keeps the destination's own pixel
    dep = np.full((6, 50), 200, np.uint8)
    gL, gR, _ = oracle_mod.synthesize_gather(f, 12, depth=dep, r=0)
    fw = oracle_mod.synthesize(f, 12, depth=dep, r=0)
    _, oL, oR = oracle_mod.disparity_lut(12)
    a, b = int(oL[200]), int(-oR[200])  # 5 and 4
    assert np.array_equal(gL[:, a:], fw.L[:, a:]) and np.array_equal(gL[:, :a], f[:, :a])
    assert np.array_equal(gR[:, :50 - b], fw.R[:, :50 - b]) and np.array_equal(gR[:, 50 - b:], f[:, 50 - b:])


# --------------------------------------- block-iterative inpainting
@pytest.mark.parametrize("seed", range(8))
def test_inpaint_blocks_brute_force(oracle_mod, seed):
    rng = np.random.default_rng(500 + seed)
    h, w = int(rng.integers(1, 9)), int(rng.integers(1, 14))
    f = rng.integers(0, 256, (h, w, 3), dtype=np.uint8)
    warp = np.where(rng.random((h, w)) < 0.45, -1, rng.integers(0, w, (h, w))).astype(np.int32)
    got, _ = oracle_mod.inpaint_blocks(f, warp)
    want = np.array(brute.inpaint_blocks(f.tolist(), warp.tolist()), np.uint8).reshape(h, w, 3)
    assert np.array_equal(got, want)


def test_inpaint_blocks_closed_forms(oracle_mod):
    rng = np.random.default_rng(8)
    f = rng.integers(0, 256, (5, 9, 3), dtype=np.uint8)
    ident = np.tile(np.arange(9, dtype=np.int32), (5, 1))
    # no holes: the warped view itself
    v, sweeps = oracle_mod.inpaint_blocks(f, ident)
    assert np.array_equal(v, f) and sweeps == 0
    # a single hole inside a constant image takes the constant in one sweep
    c = np.full((5, 9, 3), 90, np.uint8)
    wp = ident.copy()
    wp[2, 4] = -1
    v, sweeps = oracle_mod.inpaint_blocks(c, wp)
    assert np.array_equal(v, c) and sweeps == 1
    # a 1-row frame: a hole with one undamaged neighbour is never filled and
    # keeps its source pixel; one between two valid pixels takes their mean
    row = np.array([[[10, 0, 0], [20, 0, 0], [30, 0, 0], [71, 0, 0]]], np.uint8)
    v, _ = oracle_mod.inpaint_blocks(row, np.array([[-1, 1, -1, 3]], np.int32))
    assert v[0, 0].tolist() == [10, 0, 0] and v[0, 2].tolist() == [46, 0, 0]  # (20 + 71 + 1) // 2
    v, _ = oracle_mod.inpaint_blocks(row, np.array([[0, -1, -1, 3]], np.int32))
    assert v[0, 1].tolist() == [20, 0, 0] and v[0, 2].tolist() == [30, 0, 0]
    # a vertical 2-px-wide hole band in a 3-row frame fills from both sides in one sweep
    band = np.tile(np.arange(6, dtype=np.int32), (3, 1))
    band[:, 2:4] = -1
    v, sweeps = oracle_mod.inpaint_blocks(f[:3, :6], band)
    assert sweeps == 1
    top = [f[0, 1], f[1, 1]]
    assert v[0, 2].tolist() == [int((int(top[0][k]) + int(top[1][k]) + 1) // 2) for k in range(3)]


@pytest.mark.parametrize("w,h,K,threads", [(333, 191, 0, 3), (640, 360, 0, 8), (97, 64, 2, 5), (24, 9, 4, 16)])
def test_row_parallel_equals_single_thread(oracle_mod, w, h, K, threads):
    """The CPU baseline's row-parallel mode splits only row-independent
    stages: its outputs equal the single-thread oracle's for any band split."""
    frame = synth.gen_frame(31 + w, w, h, 12, 4.0)
    B = synth.default_disparity(w)
    one = oracle_mod.synthesize_views(frame, B, K=K)
    many = oracle_mod.synthesize_views_mt(frame, B, threads, K=K)
    for a, b in zip(one, many):
        assert np.array_equal(a, b)
