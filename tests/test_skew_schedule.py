"""The skewed pair schedule on the CPU (no GPU): a step-by-step model of the
tiles the score pass launches -- lane g of band b covers, in chunk c, columns
[c*wc - b*kr - g, +wc) (kr = K rounded up to 16), band b's chunks run from
floor(b*kr / wc) to ceil((n + b*kr + K - 1) / wc) - 1, tile (b, c) runs on
anti-diagonal b + c -- with the kernel's boundary buffers updated in place
(rowbuf per column, colbuf per row, carry per row block).  Each launch reads
the buffers as they were before it and applies its writes after it; the test
fails if two tiles of one launch write the same entry, if a tile reads an
entry another tile of the same launch writes, or if a tile reads an entry no
earlier launch wrote.  The model's score must equal the oracle's."""
import numpy as np
import pytest

import oracle

PAD = 32


def _model_score(q, s, sm, go, ge, R, K, wc):
    m, n = len(q), len(s)
    nbr = -(-m // R)
    nb = -(-nbr // K)
    kr = -(-K // 16) * 16
    c_lo = lambda b: b * kr // wc
    c_hi = lambda b: -(-(n + b * kr + K - 1) // wc) - 1

    def prof(row, code):
        if row >= m or code == PAD:
            return -10 ** 6
        return int(sm[q[row]][code]) + go

    rowbuf, colbuf, carry = {}, {}, {}
    best = 0
    for d in range(nb + c_hi(nb - 1)):
        tiles = [(b, d - b) for b in range(nb) if c_lo(b) <= d - b <= c_hi(b)]
        if not tiles:
            continue
        snap = {"row": dict(rowbuf), "col": dict(colbuf), "carry": dict(carry)}
        reads, writes, pend = {}, {}, []

        def rd(buf, key, t):
            reads.setdefault((buf, key), set()).add(t)
            assert key in snap[buf], f"read of an entry never written: {buf}[{key}]"
            return snap[buf][key]

        for t, (b, c) in enumerate(tiles):
            lanes = []
            for g in range(K):
                rb = b * K + g
                j0 = c * wc - b * kr - g
                has_left = 1 <= j0 <= n            # this lane computed column j0 - 1 before
                if has_left:
                    Y = [rd("col", rb * R + r, t)[0] for r in range(R)]
                    E = [snap["col"][rb * R + r][1] for r in range(R)]
                    yb, fb, yd = rd("carry", rb, t)
                else:
                    Y, E, yb, fb, yd = [-go] * R, [0] * R, -go, 0, -go
                lanes.append({"rb": rb, "j0": j0, "Y": Y, "E": E, "yd": yd, "yb": yb, "fb": fb, "S": 0})
            for st in range(wc):
                prev = [(L["yb"], L["fb"]) for L in lanes]   # what the DPP shift hands down
                for g, L in enumerate(lanes):
                    j = L["j0"] + st
                    if not 0 <= j < n:
                        continue
                    if g == 0:
                        yt, ft = rd("row", j, t) if b > 0 else (-go, 0)
                    else:
                        yt, ft = prev[g - 1]
                    dg, L["yd"] = L["yd"], yt
                    hup, F = yt, ft
                    for r in range(R):
                        tt = dg + prof(L["rb"] * R + r, int(s[j]))
                        e = max(L["E"][r] - ge, L["Y"][r], 0)
                        F = max(F - ge, hup)
                        h = max(tt, e, F)
                        L["S"] = max(L["S"], h)
                        dg, hup = L["Y"][r], h - go
                        L["Y"][r], L["E"][r] = hup, e
                    L["yb"], L["fb"] = hup, F
                    if g == K - 1 and b < nb - 1:
                        writes.setdefault(("row", j), set()).add(t)
                        pend.append((rowbuf, j, (hup, F)))
            for L in lanes:
                best = max(best, L["S"])
                for r in range(R):
                    writes.setdefault(("col", L["rb"] * R + r), set()).add(t)
                    pend.append((colbuf, L["rb"] * R + r, (L["Y"][r], L["E"][r])))
                writes.setdefault(("carry", L["rb"]), set()).add(t)
                pend.append((carry, L["rb"], (L["yb"], L["fb"], L["yd"])))
        for key, ws in writes.items():
            assert len(ws) == 1, f"two tiles of launch {d} write {key}"
            assert not (reads.get(key, set()) - ws), f"launch {d}: {key} read by one tile, written by another"
        for buf, key, v in pend:
            buf[key] = v
    return best


@pytest.mark.parametrize("K", [1, 2, 8, 16, 32])
@pytest.mark.parametrize("seed", range(8))
def test_skewed_schedule_matches_oracle(K, seed):
    rng = np.random.default_rng(seed * 7 + K)
    m, n = int(rng.integers(1, 160)), int(rng.integers(1, 140))
    R = int(rng.choice([2, 4, 8]))
    wc = int(rng.choice([16, 32, 48]))
    q = rng.integers(0, 4, m)
    s = rng.integers(0, 4, n)
    k = min(m, n)
    s[:k] = np.where(rng.random(k) < 0.7, q[:k], s[:k])      # homologous prefix
    sm = np.full((32, 32), -3, dtype=np.int32)
    for i in range(4):
        sm[i, i] = 2 + i
    go, ge = int(rng.integers(0, 6)), int(rng.integers(0, 3))
    exp = oracle.score(q.astype(np.uint8), s.astype(np.uint8), sm, go, ge)
    assert _model_score(q, s, sm, go, ge, R, K, wc) == exp, (m, n, R, K, wc, go, ge)
