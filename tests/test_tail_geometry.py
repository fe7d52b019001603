"""Index geometry of the tail kernel, checked on the CPU.

The tail kernel runs the last n levels of a transform inside LDS on
kTailS x kTailS tiles plus a recompute halo.  Its correctness rests on
index facts that this test walks exhaustively for many level sizes, using
the same region, range and fold formulas as the kernel:

* every folded read of a level's input lands inside that level's LDS region
  on a slot that was written (a loaded pixel, or an LL value the previous
  level produced);
* every predict value the update reads was computed;
* LL values written for the next level land inside its region;
* the LDS arrays fit kTailLds;
* every coefficient of every tail level is written by exactly one tile.
"""
import random

import pytest

K_TAIL_S = 64
K_TAIL_LDS = 17024


def fold(p, n):
    if 0 <= p < n:
        return p
    m = 2 * (n - 1)
    p %= m
    return m - p if p >= n else p


def fold_near(p, n):
    q = -p if p < 0 else p
    q = 2 * (n - 1) - q if q > n - 1 else q
    return -q if q < 0 else q


def test_fold_near_matches_fold():
    for n in range(2, 40):
        for p in range(-2, n + 2):
            assert fold_near(p, n) == fold(p, n), (p, n)


def halo(n, m):
    return (2 << (n - m)) - 2


def sizes_from(w0, h0, n):
    ws, hs = [w0], [h0]
    for _ in range(n):
        ws.append((ws[-1] + 1) // 2)
        hs.append((hs[-1] + 1) // 2)
    return ws, hs


def walk(w0, h0, n):
    W, H = sizes_from(w0, h0, n)
    tiles_x, tiles_y = -(-w0 // K_TAIL_S), -(-h0 // K_TAIL_S)
    lds = sum(((K_TAIL_S >> m) + 2 * halo(n, m)) ** 2 for m in range(n))
    NP = (K_TAIL_S >> 1) + 2 * halo(n, 1) + 1
    assert lds + 3 * NP * NP <= K_TAIL_LDS
    owner = [dict() for _ in range(n)]       # level m: output key -> tile
    for ty in range(tiles_y):
        for tx in range(tiles_x):
            r = halo(n, 0)
            ox, oy, N = tx * K_TAIL_S - r, ty * K_TAIL_S - r, K_TAIL_S + 2 * r
            written = {(gx, gy) for gy in range(max(oy, 0), min(oy + N, H[0]))
                       for gx in range(max(ox, 0), min(ox + N, W[0]))}
            for m in range(n):
                r = halo(n, m)
                ox, oy, N = tx * (K_TAIL_S >> m) - r, ty * (K_TAIL_S >> m) - r, (K_TAIL_S >> m) + 2 * r

                def slot(gx, gy):
                    # the kernel's division-free fold covers [-2, size + 1]
                    assert -2 <= gx <= W[m] + 1 and -2 <= gy <= H[m] + 1, (w0, h0, n, m, gx, gy)
                    assert fold_near(gx, W[m]) == fold(gx, W[m]) and fold_near(gy, H[m]) == fold(gy, H[m])
                    fx, fy = fold(gx, W[m]), fold(gy, H[m])
                    assert 0 <= fx - ox < N and 0 <= fy - oy < N, (w0, h0, n, m, tx, ty, gx, gy)
                    assert (fx, fy) in written, (w0, h0, n, m, tx, ty, gx, gy)

                rn = halo(n, m + 1) if m + 1 < n else 0
                S1 = K_TAIL_S >> (m + 1)
                cx, cy = tx * S1, ty * S1
                ns_w, ns_h, nd_w, nd_h = (W[m] + 1) // 2, (H[m] + 1) // 2, W[m] // 2, H[m] // 2
                ux0, ux1 = max(cx - rn, 0), min(cx + S1 + rn, ns_w)
                uy0, uy1 = max(cy - rn, 0), min(cy + S1 + rn, ns_h)
                px0, py0 = ux0 - 1, uy0 - 1
                assert ux1 - px0 <= NP and uy1 - py0 <= NP
                predicted = set()
                for qy in range(py0, uy1):
                    for qx in range(px0, ux1):
                        for dy in range(3):
                            for dx in range(3):
                                slot(2 * qx + dx, 2 * qy + dy)
                        predicted.add((qx, qy))
                nxt = set()
                Nn, oxn, oyn = S1 + 2 * rn, cx - rn, cy - rn
                for qy in range(uy0, uy1):
                    for qx in range(ux0, ux1):
                        slot(2 * qx, 2 * qy)
                        for (a, b) in ((qx - 1, qy), (qx, qy - 1), (qx - 1, qy - 1), (qx, qy)):
                            assert (a, b) in predicted
                        if m + 1 < n:
                            assert 0 <= qy - oyn < Nn and 0 <= qx - oxn < Nn
                            nxt.add((qx, qy))
                        if cx <= qx < cx + S1 and cy <= qy < cy + S1:
                            keys = [("hl", qx, qy)] if qx < nd_w else []
                            if qy < nd_h:
                                keys.append(("lh", qx, qy))
                                if qx < nd_w:
                                    keys.append(("hh", qx, qy))
                            if m + 1 == n:
                                keys.append(("ll", qx, qy))
                            for key in keys:
                                assert key not in owner[m], (w0, h0, n, m, key)
                                owner[m][key] = (tx, ty)
                written = nxt
    # every coefficient of every level written once
    for m in range(n):
        ns_w, ns_h, nd_w, nd_h = (W[m] + 1) // 2, (H[m] + 1) // 2, W[m] // 2, H[m] // 2
        want = ns_h * nd_w + nd_h * ns_w + nd_h * nd_w + (ns_w * ns_h if m + 1 == n else 0)
        assert len(owner[m]) == want, (w0, h0, n, m)


CASES = [(2, 2, 1), (4, 4, 2), (5, 3, 2), (64, 64, 3), (65, 65, 3), (66, 127, 3), (128, 128, 3),
         (1024, 1024, 3), (1023, 1025, 2), (130, 9, 2), (200, 17, 3), (17, 300, 3), (8, 8, 3), (9, 15, 3)]


@pytest.mark.parametrize("w0,h0,n", [c for c in CASES if c[2] >= 2])
def test_tail_geometry_listed(w0, h0, n):
    W, H = sizes_from(w0, h0, n)
    assert min(W[:n]) >= 2 and min(H[:n]) >= 2
    walk(w0, h0, n)


def test_tail_geometry_random():
    rng = random.Random(17)
    done = 0
    while done < 25:
        n = rng.choice([2, 3])
        w0, h0 = rng.randint(2, 400), rng.randint(2, 400)
        W, H = sizes_from(w0, h0, n)
        if min(W[:n]) < 2 or min(H[:n]) < 2:
            continue
        walk(w0, h0, n)
        done += 1


# ------------------------------------------------------------- inverse tail

def band_idx(q, n, par):
    return (fold(2 * q + par, n) - par) >> 1


def inv_ranges(d0, d1, n_levels, sizes):
    """Per level m (0 = finest), the needed output pixel range [d0, d1) and
    the quadruple range [q0, q1] on one axis.  Level m + 1 must produce the
    LL pixels the update at [q0, q1 + 1] reads through the fold: from
    min(q0, fold of q1 + 1) (the fold decreases past the edge) to
    min(q1 + 2, sizes[m + 1])."""
    out = []
    for m in range(n_levels):
        q0, q1 = d0 >> 1, (d1 - 1) >> 1
        out.append((d0, d1, q0, q1))
        d0, d1 = min(q0, band_idx(q1 + 1, sizes[m], 0)), min(q1 + 2, sizes[m + 1])
    out.append((d0, d1, None, None))         # LL range of the coarsest level, read from the packed array
    return out


def walk_inv(w0, h0, n):
    W, H = sizes_from(w0, h0, n)
    tiles_x, tiles_y = -(-w0 // K_TAIL_S), -(-h0 // K_TAIL_S)
    E = K_TAIL_S // 2 + 2                      # largest coefficient range per axis
    assert 8 * E * E <= K_TAIL_LDS
    written0 = {}
    for ty in range(tiles_y):
        for tx in range(tiles_x):
            rx = inv_ranges(tx * K_TAIL_S, min(tx * K_TAIL_S + K_TAIL_S, w0), n, W)
            ry = inv_ranges(ty * K_TAIL_S, min(ty * K_TAIL_S + K_TAIL_S, h0), n, H)
            produced = None                  # LL pixels the coarser level produced (level m's LL input)
            for m in reversed(range(n)):
                d0x, d1x, q0x, q1x = rx[m]
                d0y, d1y, q0y, q1y = ry[m]
                assert q1x - q0x + 3 <= E and q1y - q0y + 3 <= E
                # LL range this level reads (stored in an E x E array)
                assert rx[m + 1][1] - rx[m + 1][0] <= E and ry[m + 1][1] - ry[m + 1][0] <= E
                for (q, size, par) in [(q, W[m], p) for q in range(q0x - 1, q1x + 2) for p in (0, 1)] + \
                        [(q, H[m], p) for q in range(q0y - 1, q1y + 2) for p in (0, 1)]:
                    assert -2 <= 2 * q + par <= size + 2, (w0, h0, n, m, q)
                    assert fold_near(2 * q + par, size) == fold(2 * q + par, size)
                # LL reads of the inverse update at [q0, q1 + 1]
                for qy in range(q0y, q1y + 2):
                    for qx in range(q0x, q1x + 2):
                        ly, lx = band_idx(qy, H[m], 0), band_idx(qx, W[m], 0)
                        if m + 1 < n:
                            assert (lx, ly) in produced, (w0, h0, n, m, qx, qy)
                            d0n_x, d1n_x = rx[m + 1][0], rx[m + 1][1]
                            d0n_y, d1n_y = ry[m + 1][0], ry[m + 1][1]
                            assert d0n_x <= lx < d1n_x and d0n_y <= ly < d1n_y
                        else:
                            assert rx[n][0] <= lx < rx[n][1] and ry[n][0] <= ly < ry[n][1]
                            assert 0 <= lx < W[m + 1] and 0 <= ly < H[m + 1]
                # this level's output pixels
                out = {(x, y) for y in range(2 * q0y, 2 * q1y + 2) for x in range(2 * q0x, 2 * q1x + 2)
                       if d0x <= x < d1x and d0y <= y < d1y}
                assert len(out) == (d1x - d0x) * (d1y - d0y)
                if m == 0:
                    for p in out:
                        assert p not in written0
                        written0[p] = (tx, ty)
                produced = out
    assert len(written0) == w0 * h0


@pytest.mark.parametrize("w0,h0,n", [(16, 16, 3), (17, 33, 3), (64, 64, 3), (65, 65, 3), (130, 200, 3),
                                     (1024, 1024, 3), (8, 9, 2), (127, 66, 2), (300, 17, 2)])
def test_inverse_tail_geometry(w0, h0, n):
    W, H = sizes_from(w0, h0, n)
    assert min(W[:n]) >= 4 and min(H[:n]) >= 4
    walk_inv(w0, h0, n)


def test_inverse_tail_geometry_random():
    rng = random.Random(29)
    done = 0
    while done < 25:
        n = rng.choice([2, 3])
        w0, h0 = rng.randint(4, 400), rng.randint(4, 400)
        W, H = sizes_from(w0, h0, n)
        if min(W[:n]) < 4 or min(H[:n]) < 4:
            continue
        walk_inv(w0, h0, n)
        done += 1


def test_fold_near_covers_the_inverse_range():
    for n in range(4, 40):
        for p in range(-2, n + 3):
            assert fold_near(p, n) == fold(p, n), (p, n)


# ------------------------------------------------------------- adjoint tail

def adj_ranges(d0, d1, n_levels, sizes):
    """Adjoint tail, one axis: output pixels [d0, d1) of level m need
    quadruples [q0, q1], the transposed update at [q0 - 1, q1], coefficients
    at [q0 - 1, q1 + 1] (zero outside the bands: nothing folds) and LL pixels
    [max(q0 - 1, 0), min(q1 + 2, sizes[m + 1])) from the coarser level."""
    out = []
    for m in range(n_levels):
        q0, q1 = d0 >> 1, (d1 - 1) >> 1
        out.append((d0, d1, q0, q1))
        d0, d1 = max(q0 - 1, 0), min(q1 + 2, sizes[m + 1])
    out.append((d0, d1, None, None))
    return out


def walk_adj(w0, h0, n):
    W, H = sizes_from(w0, h0, n)
    tiles_x, tiles_y = -(-w0 // K_TAIL_S), -(-h0 // K_TAIL_S)
    E = K_TAIL_S // 2 + 2
    written0 = {}
    for ty in range(tiles_y):
        for tx in range(tiles_x):
            rx = adj_ranges(tx * K_TAIL_S, min(tx * K_TAIL_S + K_TAIL_S, w0), n, W)
            ry = adj_ranges(ty * K_TAIL_S, min(ty * K_TAIL_S + K_TAIL_S, h0), n, H)
            produced = None
            for m in reversed(range(n)):
                d0x, d1x, q0x, q1x = rx[m]
                d0y, d1y, q0y, q1y = ry[m]
                assert q1x - q0x + 3 <= E and q1y - q0y + 3 <= E
                assert rx[m + 1][1] - rx[m + 1][0] <= E and ry[m + 1][1] - ry[m + 1][0] <= E
                ns_w, ns_h = W[m + 1], H[m + 1]
                for qy in range(q0y - 1, q1y + 2):
                    for qx in range(q0x - 1, q1x + 2):
                        if 0 <= qx < ns_w and 0 <= qy < ns_h:   # an LL read that is not a zero
                            if m + 1 < n:
                                assert (qx, qy) in produced, (w0, h0, n, m, qx, qy)
                            assert rx[m + 1][0] <= qx < rx[m + 1][1] and ry[m + 1][0] <= qy < ry[m + 1][1]
                out = {(x, y) for y in range(2 * q0y, 2 * q1y + 2) for x in range(2 * q0x, 2 * q1x + 2)
                       if d0x <= x < d1x and d0y <= y < d1y}
                assert len(out) == (d1x - d0x) * (d1y - d0y)
                if m == 0:
                    for p in out:
                        assert p not in written0
                        written0[p] = (tx, ty)
                produced = out
    assert len(written0) == w0 * h0


@pytest.mark.parametrize("w0,h0,n", [(4, 4, 2), (5, 3, 2), (16, 16, 3), (65, 65, 3), (130, 200, 3),
                                     (1024, 1024, 3), (9, 15, 3), (300, 17, 2)])
def test_adjoint_tail_geometry(w0, h0, n):
    walk_adj(w0, h0, n)
