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
