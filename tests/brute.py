"""Pure-Python brute force of the pseudo-stereo pipeline, for tiny frames.

An independent restatement of each stage used to pin the C oracle: it is
written in a different form wherever the definition allows one (breadth-first
search for the region components instead of label propagation, an exact
rational rounding for the parallax, a per-destination search over all sources
instead of a scatter, linear searches for the hole neighbours).  Plain lists
and ints only; quadratic or worse, so use frames of a few hundred pixels.
"""
from __future__ import annotations

import math
from collections import deque
from fractions import Fraction


def round_half_up(q: Fraction) -> int:
    return math.floor(q + Fraction(1, 2))


def luma(r: int, g: int, b: int) -> int:
    # BT.601 luma 0.299 R + 0.587 G + 0.114 B with Q8 weights 77/150/29.
    return round_half_up(Fraction(77 * r + 150 * g + 29 * b, 256))


def weight_tables(radius: int = 3):
    ws = [round_half_up(Fraction(255) * Fraction(math.exp(-k / 4.5))) for k in range(2 * radius * radius + 1)]
    wr = [round_half_up(Fraction(255) * Fraction(math.exp(-d * d / 288.0))) for d in range(256)]
    return ws, wr


def parallax(B: int, T: int, D: int):
    """(P, oL, oR): signed total parallax and per-view shifts for depth D."""
    crossed = D > T
    m = D if crossed else 255 - D
    P = round_half_up(Fraction(B * m, 255))
    left, right = (P + 1) // 2, P // 2        # left view gets the odd pixel
    s = 1 if crossed else -1
    return s * P, s * left, -s * right


def pipeline(frame, B, T=150, K=8, g=24, tau=24, r=2, depth=None):
    """frame: list of rows of (R, G, B) tuples.  Returns a dict of stages."""
    h, w = len(frame), len(frame[0])
    Y = [[luma(*frame[y][x]) for x in range(w)] for y in range(h)]
    gw, gh = -(-w // K), -(-h // K)

    def ramp(row):
        # row ramp: far (0) at the top block row, near (255) at the bottom
        return 0 if gh == 1 else round_half_up(Fraction(255 * row, gh - 1))

    if depth is None:
        # block means and edge flags
        mean, edge = {}, {}
        for by in range(gh):
            for bx in range(gw):
                pix = [(x, y) for y in range(by * K, min(by * K + K, h))
                       for x in range(bx * K, min(bx * K + K, w))]
                n = len(pix)
                mean[bx, by] = tuple(round_half_up(Fraction(sum(frame[y][x][c] for x, y in pix), n))
                                     for c in range(3))
                e = False
                for x, y in pix:
                    if x + 1 < w and abs(Y[y][x + 1] - Y[y][x]) > g:
                        e = True
                    if y + 1 < h and abs(Y[y + 1][x] - Y[y][x]) > g:
                        e = True
                edge[bx, by] = e

        def linked(a, b):
            if edge[a] or edge[b]:
                return False
            return sum(abs(mean[a][c] - mean[b][c]) for c in range(3)) <= tau

        # components by breadth-first search; label = smallest block index
        comp = {}
        for start in sorted(mean, key=lambda p: p[1] * gw + p[0]):
            if start in comp:
                continue
            members, q = [start], deque([start])
            comp[start] = None
            while q:
                bx, by = q.popleft()
                for nx, ny in ((bx + 1, by), (bx - 1, by), (bx, by + 1), (bx, by - 1)):
                    if 0 <= nx < gw and 0 <= ny < gh and (nx, ny) not in comp and linked((bx, by), (nx, ny)):
                        comp[nx, ny] = None
                        members.append((nx, ny))
                        q.append((nx, ny))
            lab = min(by * gw + bx for bx, by in members)
            for m in members:
                comp[m] = (lab, members)
        labels = [[comp[bx, by][0] for bx in range(gw)] for by in range(gh)]
        # background: largest non-edge region, ties to the smaller label
        regions = {}
        for (bx, by), (lab, members) in comp.items():
            if not edge[bx, by]:
                regions[lab] = members
        bg = None
        if regions:
            bg = min(regions, key=lambda l: (-len(regions[l]), l))
        dblk = {}
        for (bx, by), (lab, members) in comp.items():
            if edge[bx, by] or lab == bg:
                dblk[bx, by] = ramp(by)
            else:
                dblk[bx, by] = ramp(max(my for _, my in members))
        D0 = [[0] * w for _ in range(h)]
        for y in range(h):
            for x in range(w):
                bx, by = x // K, y // K
                if not edge[bx, by]:
                    D0[y][x] = dblk[bx, by]
                    continue
                cands = []
                for dy in (-1, 0, 1):
                    for dx in (-1, 0, 1):
                        c = (bx + dx, by + dy)
                        if c in mean and not edge[c]:
                            d = sum(abs(frame[y][x][ch] - mean[c][ch]) for ch in range(3))
                            cands.append((d, (dy + 1) * 3 + (dx + 1), c))
                D0[y][x] = dblk[min(cands)[2]] if cands else ramp(by)
        stats = [[mean[bx, by][0] | mean[bx, by][1] << 8 | mean[bx, by][2] << 16 | int(edge[bx, by]) << 24
                  for bx in range(gw)] for by in range(gh)]
        dblk_grid = [[dblk[bx, by] for bx in range(gw)] for by in range(gh)]
    else:
        D0 = [list(row) for row in depth]
        labels = stats = dblk_grid = None

    ws, wr = weight_tables(max(r, 1))
    Df = [[0] * w for _ in range(h)]
    for y in range(h):
        for x in range(w):
            num = den = 0
            for qy in range(max(0, y - r), min(h, y + r + 1)):
                for qx in range(max(0, x - r), min(w, x + r + 1)):
                    wt = ws[(qx - x) ** 2 + (qy - y) ** 2] * wr[abs(Y[qy][qx] - Y[y][x])]
                    num += wt * D0[qy][qx]
                    den += wt
            Df[y][x] = round_half_up(Fraction(num, den))

    views = {}
    for vi, name in enumerate("LR"):
        warp = [[-1] * w for _ in range(h)]
        src = [[-1] * w for _ in range(h)]
        for y in range(h):
            # per destination: every source of the row that lands on it
            for xd in range(w):
                hits = [(Df[y][x], x) for x in range(w)
                        if x + parallax(B, T, Df[y][x])[1 + vi] == xd]
                if hits:
                    warp[y][xd] = max(hits)[1]
            for xd in range(w):
                if warp[y][xd] >= 0:
                    src[y][xd] = warp[y][xd]
                    continue
                left = [j for j in range(xd) if warp[y][j] >= 0]
                right = [j for j in range(xd + 1, w) if warp[y][j] >= 0]
                if not left and not right:
                    src[y][xd] = xd
                    continue
                opts = []
                if left:
                    j = left[-1]
                    opts.append((Df[y][warp[y][j]], 0 if name == "L" else 1, warp[y][j]))
                if right:
                    j = right[0]
                    opts.append((Df[y][warp[y][j]], 1 if name == "L" else 0, warp[y][j]))
                src[y][xd] = min(opts)[2]
        img = [[frame[y][src[y][x]] for x in range(w)] for y in range(h)]
        views[name] = (img, warp, src)
    L, R = views["L"][0], views["R"][0]
    A = [[(L[y][x][0], R[y][x][1], R[y][x][2]) for x in range(w)] for y in range(h)]
    return {"Y": Y, "D0": D0, "Df": Df, "labels": labels, "stats": stats, "dblk": dblk_grid,
            "L": L, "R": R, "A": A,
            "warpL": views["L"][1], "warpR": views["R"][1],
            "srcL": views["L"][2], "srcR": views["R"][2]}


def hsbs(L, R):
    """Half side-by-side frame, pixel by pixel: half p of a view = mean of its
    columns 2p and 2p+1 rounded half up (only column 2p if 2p+1 is past the
    edge); left half = left view, floor(w/2) columns; right half = right view,
    the remaining columns."""
    h, w = len(L), len(L[0])
    hw = w // 2
    out = [[None] * w for _ in range(h)]
    for y in range(h):
        for x in range(w):
            view, p = (L, x) if x < hw else (R, x - hw)
            a = view[y][2 * p]
            b = view[y][2 * p + 1] if 2 * p + 1 < w else a
            out[y][x] = tuple(round_half_up(Fraction(a[c] + b[c], 2)) for c in range(3))
    return out


def gather(frame, Df, B, T=150):
    """Fig. 3 gather, pixel by pixel: L(x) = I(x - oL(Df(x))), R(x) =
    I(x - oR(Df(x))), falling back to I(x) outside the row; A = (L.R, R.G, R.B)."""
    h, w = len(frame), len(frame[0])
    L = [[None] * w for _ in range(h)]
    R = [[None] * w for _ in range(h)]
    A = [[None] * w for _ in range(h)]
    for y in range(h):
        for x in range(w):
            _, oL, oR = parallax(B, T, Df[y][x])
            xl, xr = x - oL, x - oR
            xl = xl if 0 <= xl < w else x
            xr = xr if 0 <= xr < w else x
            L[y][x] = tuple(frame[y][xl])
            R[y][x] = tuple(frame[y][xr])
            A[y][x] = (L[y][x][0], R[y][x][1], R[y][x][2])
    return L, R, A


def inpaint_blocks(frame, warp):
    """Block-iterative inpainting, written out: damaged = warp < 0; Jacobi
    sweeps fill every damaged pixel with >= 2 undamaged 8-neighbours by their
    rounded-half-up mean; stop when a sweep fills nothing; leftovers keep the
    source pixel."""
    h, w = len(warp), len(warp[0])
    dmg = [[warp[y][x] < 0 for x in range(w)] for y in range(h)]
    col = [[(0, 0, 0) if warp[y][x] < 0 else tuple(frame[y][warp[y][x]]) for x in range(w)] for y in range(h)]
    while True:
        upd = {}
        for y in range(h):
            for x in range(w):
                if not dmg[y][x]:
                    continue
                nb = [col[yy][xx] for yy in range(y - 1, y + 2) for xx in range(x - 1, x + 2)
                      if (yy, xx) != (y, x) and 0 <= yy < h and 0 <= xx < w and not dmg[yy][xx]]
                if len(nb) >= 2:
                    upd[(y, x)] = tuple(round_half_up(Fraction(sum(c[k] for c in nb), len(nb))) for k in range(3))
        if not upd:
            break
        for (y, x), c in upd.items():
            col[y][x] = c
            dmg[y][x] = False
    return [[tuple(frame[y][x]) if dmg[y][x] else col[y][x] for x in range(w)] for y in range(h)]
