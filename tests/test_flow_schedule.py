"""CPU model of the pipelined ("flow") pass over one long pair, checked
against the oracle before and beside the HIP kernel (no GPU needed).

The flow pass gives every wavefront one band of 64 lanes x R query rows at a
time; the wave sweeps all subject columns, lane g one column behind lane
g - 1 (the DPP pipeline of the tile kernels).  The band's last lane hands its
bottom row (H - Go and F per column) to the band below through one 64-bit
word per column, updated in place: bits 0-23 hold H - Go + Go, bits 24-47
F + Go, bits 48-63 a tag, band + 1 (bands number at most 2^16, the buffer
is zeroed per call).  A reader polls a word until its tag names the band just
above; any other word -- zero, or a band further up -- is rejected, so no
progress assumption is needed.  The values fit 24 bits when the largest
score, max(SM) x min(m, n), is below 2^24 (the host checks this before it
picks the flow pass).  Waves take bands w, w + G, w + 2G, ... in order.

The model runs the waves as interleaved step machines under random
schedules, including schedules that stall bands, with words carried through
the same packing; it checks that every accepted read returns the value the
band above wrote for that column, that no word is overwritten before its
reader consumed it, and that the score equals the oracle's.  It also checks
the kernel's address bounds (buffer entries, subject blocks, profile row
blocks) over many shapes."""
import numpy as np
import pytest

import oracle
import synth

MASK24 = (1 << 24) - 1


def pack(y, f, go, tag):
    assert 0 <= y + go <= MASK24 and 0 <= f + go <= MASK24 and 0 <= tag < (1 << 16)
    return (y + go) | ((f + go) << 24) | (tag << 48)


def unpack(w, go):
    return (w & MASK24) - go, ((w >> 24) & MASK24) - go, w >> 48


class Band:
    """One wavefront sweeping one band: lane g computes column t - g at step t."""

    def __init__(self, b, q, d, sm, go, ge, R, K=64):
        self.b, self.q, self.d, self.sm, self.go, self.ge, self.R, self.K = b, q, d, sm, go, ge, R, K
        self.m, self.n = len(q), len(d)
        self.t = 0
        self.T = self.n + K - 1
        self.Y = [[-go] * R for _ in range(K)]
        self.E = [[0] * R for _ in range(K)]
        self.ydiag = [-go] * K
        self.ybot = [-go] * K
        self.fbot = [0] * K
        self.S = 0

    def done(self):
        return self.t >= self.T

    def row(self, g, r):
        return (self.b * self.K + g) * self.R + r       # 0-based query row

    def step(self, top):
        """One step; top = (Y, F) of the band above at the head's column, or
        None on the matrix border.  Returns the tail lane's (column, Y, F)."""
        go, ge, K, R = self.go, self.ge, self.K, self.R
        t = self.t
        prev_ybot, prev_fbot = list(self.ybot), list(self.fbot)
        out = None
        for g in range(K):
            j = t - g
            if not (0 <= j < self.n):
                continue
            if g == 0:
                yt, ft = top if top is not None else (-go, 0)
            else:
                yt, ft = prev_ybot[g - 1], prev_fbot[g - 1]
            dg = self.ydiag[g]
            self.ydiag[g] = yt
            hup, F = yt, ft
            for r in range(R):
                i = self.row(g, r)
                # profile entry s + Go against the diagonal's H - Go; pad rows score far below
                s = int(self.sm[self.q[i], self.d[j]]) + go if i < self.m else -10**6
                tt = dg + s
                e = max(self.E[g][r] - ge, self.Y[g][r], 0)
                F = max(F - ge, hup)
                h = max(tt, e, F, 0)
                if i < self.m:
                    self.S = max(self.S, h)
                dg = self.Y[g][r]
                hup = h - go
                self.Y[g][r] = hup
                self.E[g][r] = e
            self.ybot[g], self.fbot[g] = hup, F
            if g == K - 1:
                out = (j, hup, F)
        self.t += 1
        return out


def run_flow(q, d, sm, go, ge, R, G, rng, stall=0.0, K=64, tag_check=True):
    m, n = len(q), len(d)
    nb = -(-m // (K * R))
    buf = [0] * (n + 16)                             # zeroed per call
    written = {}                                     # (band, column) -> (Y, F)
    consumed = set()
    waves = []
    for w in range(min(G, nb)):
        waves.append({"bands": list(range(w, nb, G)), "cur": None})
    S = 0
    while True:
        live = [w for w in waves if w["bands"] or w["cur"] is not None]
        if not live:
            break
        w = live[rng.integers(len(live))]
        if rng.random() < stall:
            continue
        if w["cur"] is None:
            w["cur"] = Band(w["bands"].pop(0), q, d, sm, go, ge, R, K)
        band = w["cur"]
        top = None
        j = band.t                                    # the head's column
        if band.b > 0 and j < n:
            y, f, tag = unpack(buf[j], go)
            if tag_check and tag != band.b:
                continue                              # not written yet: poll again later
            if tag_check:
                assert written[(band.b - 1, j)] == (y, f), "accepted a word of another band"
            consumed.add((band.b - 1, j))
            top = (y, f)
        out = band.step(top)
        if out is not None and band.b < nb - 1:
            jj, y, f = out
            # in place: the word replaced is the band above's, which this band read
            if band.b >= 1:
                assert (band.b - 1, jj) in consumed, "word overwritten before it was read"
            buf[jj] = pack(y, f, go, band.b + 1)
            written[(band.b, jj)] = (y, f)
        if band.done():
            S = max(S, band.S)
            w["cur"] = None
    return S


@pytest.mark.parametrize("seed", range(24))
def test_flow_model_matches_oracle(seed):
    rng = np.random.default_rng(500 + seed)
    K = int(rng.choice([4, 8, 64]))                  # narrow bands keep the model small
    R = int(rng.choice([1, 2, 4]))
    m = int(rng.integers(1, 3 * K * R + 5))
    n = int(rng.integers(1, 40))
    alpha = int(rng.choice([2, 4, 20]))
    if seed % 3 == 0:
        q = rng.integers(0, alpha, size=m).astype(np.uint8)
        d = np.concatenate([q[: n // 2], rng.integers(0, alpha, size=n - n // 2)]).astype(np.uint8)
    else:
        q = rng.integers(0, alpha, size=m).astype(np.uint8)
        d = rng.integers(0, alpha, size=n).astype(np.uint8)
    sm = synth.random_matrix(rng, -4, 5)
    go, ge = int(rng.integers(0, 8)), int(rng.integers(0, 4))
    G = int(rng.integers(1, 5))
    got = run_flow(q, d, sm, go, ge, R, G, rng, stall=float(rng.choice([0.0, 0.3])), K=K)
    assert got == oracle.score(q, d, sm, go, ge)


def run_flow_blockwise(q, d, sm, go, ge, R, G, rng, stall=0.0, K=64, slack=32, check_all=True):
    """The pass with the block-wise tag check (from 8 rows per lane on): the
    head keeps a ring of 16 words, the word of column t + 16 read (a snapshot
    of the buffer) at step t, past column n - 1 read as 0 (the range-checked
    descriptor).  At the start of a block whose columns are all inside the
    matrix the least tag of its 16 words must be the band's own b; otherwise
    the band polls until the word of column min(t0 + 15 + slack, n - 1)
    carries tag b, reads the 16 words again and checks once more.  The block
    that reaches past column n - 1 checks its words one by one (polling the
    buffer).  check_all=False checks only the block's first word."""
    m, n = len(q), len(d)
    nb = -(-m // (K * R))
    buf = [0] * (n + 16)
    written = {}
    consumed = set()
    load = lambda j: buf[j] if j < n else 0
    waves = [{"bands": list(range(w, nb, G)), "cur": None} for w in range(min(G, nb))]
    S = 0
    while True:
        live = [w for w in waves if w["bands"] or w["cur"] is not None]
        if not live:
            break
        w = live[rng.integers(len(live))]
        if rng.random() < stall:
            continue
        if w["cur"] is None:
            band = Band(w["bands"].pop(0), q, d, sm, go, ge, R, K)
            band.ring = [load(min(u, n - 1)) for u in range(16)]
            band.checked = -1
            w["cur"] = band
        band = w["cur"]
        t = band.t
        top = None
        if band.b > 0:
            t0 = t - t % 16
            whole = t0 + 15 < n
            if whole and band.checked != t0:
                tags = [unpack(x, go)[2] for x in band.ring]
                assert max(tags) <= band.b, "a word of a band below was read"
                if (min(tags) if check_all else tags[0]) < band.b:
                    if unpack(buf[min(t0 + 15 + slack, n - 1)], go)[2] != band.b:
                        continue                              # still waiting
                    band.ring = [load(t0 + u) for u in range(16)]
                    continue                                  # check the words read again
                band.checked = t0
            word = band.ring[t % 16]
            if t < n:
                y, f, tag = unpack(word, go)
                if not whole and tag != band.b:
                    y, f, tag = unpack(buf[t], go)            # poll the word itself
                    if tag != band.b:
                        continue
                if check_all:
                    assert tag == band.b and written[(band.b - 1, t)] == (y, f), "accepted a word of another band"
                consumed.add((band.b - 1, t))
                top = (y, f)
            band.ring[t % 16] = load(t + 16)                  # read ahead
        out = band.step(top)
        if out is not None and band.b < nb - 1:
            jj, y, f = out
            if band.b >= 1 and check_all:
                assert (band.b - 1, jj) in consumed, "word overwritten before it was read"
            buf[jj] = pack(y, f, go, band.b + 1)
            written[(band.b, jj)] = (y, f)
        if band.done():
            S = max(S, band.S)
            w["cur"] = None
    return S


@pytest.mark.parametrize("seed", range(24))
def test_blockwise_check_matches_oracle(seed):
    """Block-wise checks with a read-ahead ring and the resynchronising wait,
    under random and stalling schedules: every accepted word is the band
    above's for that column, no word is replaced before it was read, and the
    score equals the oracle's."""
    rng = np.random.default_rng(700 + seed)
    K = int(rng.choice([4, 8, 16]))
    R = int(rng.choice([1, 2]))
    m = int(rng.integers(1, 3 * K * R + 5))
    n = int(rng.integers(1, 70))
    alpha = int(rng.choice([2, 4, 20]))
    q = rng.integers(0, alpha, size=m).astype(np.uint8)
    h = min(n // 2, m) if seed % 3 == 0 else 0          # a homologous stretch
    d = np.concatenate([q[:h], rng.integers(0, alpha, size=n - h)]).astype(np.uint8)
    sm = synth.random_matrix(rng, -4, 5)
    go, ge = int(rng.integers(0, 8)), int(rng.integers(0, 4))
    G = int(rng.integers(1, 5))
    slack = int(rng.choice([0, 4, 32]))
    got = run_flow_blockwise(q, d, sm, go, ge, R, G, rng, stall=float(rng.choice([0.0, 0.3])), K=K, slack=slack)
    assert got == oracle.score(q, d, sm, go, ge)


def test_blockwise_model_needs_every_tag():
    """Checking only the block's first word lets later stale words through:
    the adversarial schedules then give wrong scores."""
    wrong = 0
    for seed in range(12):
        rng = np.random.default_rng(950 + seed)
        q = rng.integers(0, 4, size=40).astype(np.uint8)
        d = np.concatenate([q[5:35], rng.integers(0, 4, size=20)]).astype(np.uint8)
        sm = synth.dna_matrix(2, -3)
        got = run_flow_blockwise(q, d, sm, 3, 1, 2, 3, rng, stall=0.3, K=4, slack=0, check_all=False)
        wrong += got != oracle.score(q, d, sm, 3, 1)
    assert wrong > 0


def test_model_catches_a_missing_tag_check():
    """The schedules are adversarial enough: a reader that takes whatever
    word it finds (no tag check) reads too early and gets wrong scores."""
    wrong = 0
    for seed in range(12):
        rng = np.random.default_rng(900 + seed)
        q = rng.integers(0, 4, size=40).astype(np.uint8)
        d = np.concatenate([q[5:30], rng.integers(0, 4, size=10)]).astype(np.uint8)
        sm = synth.dna_matrix(2, -3)
        got = run_flow(q, d, sm, 3, 1, 2, 3, rng, stall=0.3, K=4, tag_check=False)
        wrong += got != oracle.score(q, d, sm, 3, 1)
    assert wrong > 0


def test_stale_words_are_rejected():
    """Whatever a word held before (zero, or a band further up), its tag is
    not the reader's expected one: tags are unique per band in a call."""
    go = 10
    for b in range(1, 300):
        expect = b
        for older in range(0, b - 1):                # bands above the one just above
            assert unpack(pack(3, 4, go, older + 1), go)[2] != expect
        assert unpack(0, go)[2] != expect             # the zeroed buffer


def test_packing_covers_the_value_range():
    go = 32000
    top = (1 << 24) - 1 - go
    for y, f in [(-go, -go), (-go, 0), (top, top), (5, -go)]:
        for tag in (1, 77, (1 << 16) - 1):
            assert unpack(pack(y, f, go, tag), go) == (y, f, tag)


@pytest.mark.parametrize("R", [4, 8, 16])
def test_flow_addresses_stay_in_bounds(R):
    """Every index the flow kernel forms stays inside its buffer: handoff
    words (n + 16 entries, the dropped sink at entry n),
    subject blocks (n_pad bytes), profile row blocks (nbr + 1)."""
    rng = np.random.default_rng(R)
    for _ in range(300):
        m, n = int(rng.integers(1, 5000)), int(rng.integers(1, 5000))
        nbr = -(-m // R)
        nb = -(-nbr // 64)
        n_pad = (n + 15) // 16 * 16 + 256
        T = n + 63
        steps = -(-T // 16) * 16
        for b in (0, nb - 1):
            for g in (0, 63):
                rb = min(b * 64 + g, nbr)
                assert 0 <= rb <= nbr
            # the head polls words j = t < n; the read-ahead and a block's
            # reloads (columns up to t0 + 31) go through a descriptor whose
            # range is the n words (a read past it returns 0 and touches no
            # memory), inside the n + 16 allocated entries; a block's wait
            # for the band above polls column min(t0 + 15 + 32, n - 1)
            assert n * 8 <= (n + 16) * 8
            for t0 in range(0, steps + 16, 16):
                jr = min(t0 + 15 + 32, n - 1)
                assert 0 <= jr < n
                blk = min(t0 + 16, n_pad - 16) // 16
                assert 0 <= blk * 16 and blk * 16 + 16 <= n_pad
            # the tail's store: column j = t - 63 in [0, n), else the dropped
            # sink offset, entry n (inside the n + 16 allocated entries)
            for t in (0, 62, 63, T - 1, steps - 1):
                j = t - 63
                off = j if 0 <= j < n else n
                assert 0 <= off <= n < n + 16
        assert nb <= (1 << 16) or m > (1 << 24)


def lap_tag(column, ring, tag):
    return (((column // ring) & 1) << 15) | (tag & 0x7FFF)


def run_flow_groups(q, d, sm, go, ge, R, W, grid, rng, stall=0.0, K=64, ring=64, block=16, check=True, lap=True,
                    wait=True):
    """The pass with workgroups of W waves: wave w of workgroup g is wave
    g * W + w and takes bands w', w' + G, ... (G = grid * W).  A band whose
    band above runs on the previous wave of its workgroup (w >= 1) reads that
    band's bottom row from a ring of `ring` tagged words in the workgroup's
    memory instead of the global buffer; its writer waits, at the start of
    each block of `block` steps, until the reader has published (at its own
    block starts) that it consumed every column the block's words would
    replace.  Progress counts columns across rounds as r * (n + ring) + column,
    and a reader publishes (r + 1) * (n + ring) when its band ends.  A ring
    word's tag holds the lap parity of its column (column // ring, bit 15)
    beside the low 15 bits of band + 1: a slot also holds the same band's word
    of a column one lap back, which the band tag alone would not tell apart."""
    m, n = len(q), len(d)
    nb = -(-m // (K * R))
    G = grid * W
    big = n + ring
    gbuf = [0] * (n + 16)
    rings = {(g, w): [0] * ring for g in range(grid) for w in range(W - 1)}     # link w -> w + 1
    slot_of = {key: [None] * ring for key in rings}                         # (band, column) held
    progress = {(g, w): 0 for g in range(grid) for w in range(1, W)}           # published by readers
    written, consumed = {}, set()
    waves = []
    for g in range(grid):
        for w in range(W):
            wid = g * W + w
            bands = list(range(wid, nb, G))
            waves.append({"g": g, "w": w, "bands": bands, "cur": None, "r": -1})
    S = 0
    while True:
        live = [x for x in waves if x["bands"] or x["cur"] is not None]
        if not live:
            break
        x = live[rng.integers(len(live))]
        if rng.random() < stall:
            continue
        if x["cur"] is None:
            x["cur"] = Band(x["bands"].pop(0), q, d, sm, go, ge, R, K)
            x["r"] += 1
        band, g, w, r = x["cur"], x["g"], x["w"], x["r"]
        t = band.t
        lds_top = w >= 1 and band.b > 0
        lds_bot = w <= W - 2 and band.b < nb - 1
        if lds_top and t % block == 0:
            progress[(g, w)] = max(progress[(g, w)], r * big + t)
        if wait and lds_bot and t % block == 0:
            # the block writes columns up to t + block - 1 - (K - 1)
            if r * big + t + block - 1 - (K - 1) - ring >= progress[(g, w + 1)]:
                continue                                  # reader too far behind: wait
        top = None
        if band.b > 0 and t < n:
            if lds_top:
                y, f, tag = unpack(rings[(g, w - 1)][t % ring], go)
                want = lap_tag(t, ring, band.b) if lap else band.b & 0x7FFF
            else:
                y, f, tag = unpack(gbuf[t], go)
                want = band.b
            if tag != want:
                continue                                  # not written yet: poll again later
            if check:
                assert written[(band.b - 1, t)] == (y, f), "accepted a word of another band"
            consumed.add((band.b - 1, t))
            top = (y, f)
        out = band.step(top)
        if out is not None and band.b < nb - 1:
            jj, y, f = out
            if lds_bot:
                key = (g, w)
                held = slot_of[key][jj % ring]
                if check and held is not None:
                    assert held in consumed, f"ring word {held} replaced before it was read"
                rings[key][jj % ring] = pack(y, f, go, lap_tag(jj, ring, band.b + 1) if lap else (band.b + 1) & 0x7FFF)
                slot_of[key][jj % ring] = (band.b, jj)
            else:
                gbuf[jj] = pack(y, f, go, band.b + 1)
            written[(band.b, jj)] = (y, f)
        if band.done():
            S = max(S, band.S)
            if lds_top:
                progress[(g, w)] = (r + 1) * big
            x["cur"] = None
    return S


@pytest.mark.parametrize("seed", range(30))
def test_flow_groups_model_matches_oracle(seed):
    """Workgroup rings under random and stalling schedules: scores equal the
    oracle's, no ring word is replaced before its reader took it, and the
    schedule never deadlocks (some wave can always move: the loop ends)."""
    rng = np.random.default_rng(700 + seed)
    K = int(rng.choice([4, 8]))
    R = int(rng.choice([1, 2]))
    W = int(rng.choice([2, 3, 4]))
    grid = int(rng.integers(1, 3))
    m = int(rng.integers(1, 4 * W * grid * K * R + 5))
    n = int(rng.integers(1, 120))
    ring = int(rng.choice([32, 40, 64]))
    q = rng.integers(0, 4, size=m).astype(np.uint8)
    d = np.concatenate([q[: n // 2], rng.integers(0, 4, size=n - n // 2)]).astype(np.uint8)
    sm = synth.dna_matrix(2, -3)
    go, ge = int(rng.integers(0, 6)), int(rng.integers(0, 3))
    got = run_flow_groups(q, d, sm, go, ge, R, W, grid, rng, stall=float(rng.choice([0.0, 0.3])), K=K,
                          ring=ring)
    assert got == oracle.score(q, d, sm, go, ge)


def test_flow_groups_model_needs_the_lap_bit():
    """Without the lap parity in the ring tags a reader ahead of its writer
    takes the same band's word of the column one lap back."""
    caught = 0
    for seed in range(12):
        rng = np.random.default_rng(800 + seed)
        q = rng.integers(0, 4, size=160).astype(np.uint8)
        d = np.concatenate([q[10:90], rng.integers(0, 4, size=60)]).astype(np.uint8)
        sm = synth.dna_matrix(2, -3)
        try:
            got = run_flow_groups(q, d, sm, 3, 1, 1, 4, 1, rng, stall=0.3, K=4, ring=32, lap=False)
            caught += got != oracle.score(q, d, sm, 3, 1)
        except (AssertionError, KeyError):
            caught += 1
    assert caught > 0


def test_flow_groups_model_catches_a_missing_wait():
    """The writer's wait is what keeps ring words alive: without it some word
    is replaced before its reader took it (or a wrong score follows)."""
    caught = 0
    for seed in range(12):
        rng = np.random.default_rng(950 + seed)
        q = rng.integers(0, 4, size=200).astype(np.uint8)
        d = np.concatenate([q[20:90], rng.integers(0, 4, size=60)]).astype(np.uint8)
        sm = synth.dna_matrix(2, -3)
        try:
            got = run_flow_groups(q, d, sm, 3, 1, 1, 3, 1, rng, stall=0.3, K=4, ring=32, wait=False)
            caught += got != oracle.score(q, d, sm, 3, 1)
        except (AssertionError, KeyError):
            caught += 1
    assert caught > 0
