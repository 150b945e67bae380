"""Host model of the index arithmetic of the table construction's split and
pack steps (the tile-level merge of Algorithm 3 with block-wise prefix sums,
Section 4.2.2), run with arbitrary merge keys.

Every address the pack kernel reads or writes is derived from tile counts and
offsets that one kernel (the tile aggregation) wrote from one reading of the
weights, plus merge keys that may be inconsistent with them (the total weight
and grid come from an earlier reading).  This model follows the kernel's
control flow at tile granularity with keys drawn at random, not sorted and not
consistent with the counts, and checks the invariants that keep every access
in range: the start of each pack block, both tile cursors, the window
indices, the tiles whose sides are fetched, and every table index written.
"""
import numpy as np
import pytest

TILE = 1024
TPB = 256  # threads per pack block
FH_NONE = -1


def pack_start(C, psteps, b, DP, EP):
    s0 = b * psteps
    lo, hi = max(0, s0 - C), min(s0, C)
    while lo < hi:
        x = (lo + hi + 1) >> 1
        y1 = s0 - x + 1
        ok = (y1 > C) or (x < C and DP[x] < EP[y1])
        if ok:
            lo = x
        else:
            hi = x - 1
    return lo


def run_block(rng, n, C, psteps, b, DP, EP, NL, PO):
    s0 = b * psteps
    s1 = min(s0 + psteps, 2 * C)
    x0 = pack_start(C, psteps, b, DP, EP)
    y0 = s0 - x0
    assert 0 <= x0 <= C and 0 <= y0 <= C
    W = psteps + 2
    dp = [DP[x0 + i] if x0 + i <= C else 2**64 - 1 for i in range(W)]
    ep = [EP[y0 + i] if y0 + i <= C else 2**64 - 1 for i in range(W)]
    nlx = [NL[min(x0 + i, C)] for i in range(W)]
    nly = [NL[min(y0 + i, C)] for i in range(W)]

    def tile_cnt(c):
        return min(TILE, n - c * TILE)

    def lights_of(c):
        if c >= C:
            return 0
        i = c - x0
        assert 0 <= i and i + 1 < W
        return nlx[i + 1] - nlx[i]

    def heavies_of(c):
        if c >= C:
            return 0
        i = c - y0
        assert 0 <= i and i + 1 < W
        return tile_cnt(c) - (nly[i + 1] - nly[i])

    written = []

    def fetch(c, first, cnt):
        if cnt == 0:
            return []
        assert 0 <= c < C and 0 <= first and first + cnt <= tile_cnt(c)
        # thread t loads slots t k .. t k + k - 1, each clamped to cnt - 1
        k = -(-cnt // TPB)
        for t in (0, TPB - 1):
            for e in range(k):
                j = min(t * k + e, cnt - 1)
                assert 0 <= first + j < tile_cnt(c)
        return [c * TILE + PO[c][first + j] for j in range(cnt)]

    # the sides staged first, and the cursors inside them (any count the
    # searches can return: they are clamped to the side)
    A = fetch(x0, 0, lights_of(x0))
    hb = heavies_of(y0)
    B = fetch(y0, tile_cnt(y0) - hb if y0 < C else 0, hb)
    pl = int(rng.integers(0, len(A) + 1))
    ph = int(rng.integers(0, len(B) + 1))
    x, y = x0, y0
    for s in range(s0, s1):
        xi, yi = x - x0, y - y0
        assert 0 <= xi and 0 <= yi and xi + 1 < W and yi + 1 < W
        has_h, has_l = y + 1 <= C, x + 1 <= C
        EPn = ep[yi + 1]
        heavy_ev = has_h and (not has_l or not (x + 1 < C and dp[x + 1 - x0] < EPn))
        assert has_h or has_l  # s < 2C: some tile event is left
        need = s + 1 < s1
        if need:
            hc = heavies_of(y + 1)  # read on either kind of event, as the kernel does
            if heavy_ev:
                nxt = fetch(y + 1, tile_cnt(y + 1) - hc if y + 1 < C else 0, hc)
            else:
                nxt = fetch(x + 1, 0, lights_of(x + 1))
        # the cell: counts from searches clamped to what is left of each side
        if heavy_ev:
            nhc = len(B) - ph
            nlc = int(rng.integers(0, len(A) - pl + 1))
        else:
            nlc = len(A) - pl
            nhc = int(rng.integers(0, len(B) - ph + 1)) if y < C else 0
        written += A[pl:pl + nlc] + B[ph:ph + nhc]
        pl += nlc
        ph += nhc
        assert pl <= len(A) and ph <= len(B)
        if heavy_ev:
            y += 1
            ph = 0
            if need:
                B = nxt
        else:
            x += 1
            pl = 0
            if need:
                A = nxt
        assert 0 <= x <= C and 0 <= y <= C
    return written


@pytest.mark.parametrize("seed", range(12))
def test_pack_indices_stay_in_range_with_arbitrary_keys(seed):
    rng = np.random.default_rng(seed)
    C = int(rng.integers(1, 40))
    n = (C - 1) * TILE + int(rng.integers(1, TILE + 1))
    psteps = int(rng.choice([4, 8, 16, 32]))
    # per-tile light counts and offsets as the tile aggregation writes them:
    # a permutation of the tile's offsets, its lights first
    cnts = [min(TILE, n - c * TILE) for c in range(C)]
    lights = [int(rng.integers(0, cnt + 1)) for cnt in cnts]
    NL = np.concatenate([[0], np.cumsum(lights)]).astype(np.int64)
    PO = [rng.permutation(cnt) for cnt in cnts]
    # merge keys from another reading of the weights: anything at all
    kind = seed % 3
    if kind == 0:
        DP = [int(v) for v in rng.integers(0, 2**63, C + 1, dtype=np.uint64)]
        EP = [int(v) for v in rng.integers(0, 2**63, C + 1, dtype=np.uint64)]
    elif kind == 1:  # wrapped 128-bit differences: huge keys
        DP = [int(v) + 2**63 for v in rng.integers(0, 2**62, C + 1, dtype=np.uint64)]
        EP = [int(v) for v in rng.integers(0, 4, C + 1, dtype=np.uint64)]
    else:  # descending
        DP = sorted((int(v) for v in rng.integers(0, 2**40, C + 1, dtype=np.uint64)), reverse=True)
        EP = sorted((int(v) for v in rng.integers(0, 2**40, C + 1, dtype=np.uint64)), reverse=True)
    npack = -(-2 * C // psteps)
    for b in range(npack):
        idx = run_block(rng, n, C, psteps, b, DP, EP, NL, PO)
        assert all(0 <= i < n for i in idx)


def test_pack_start_range_is_independent_of_keys():
    rng = np.random.default_rng(99)
    for _ in range(200):
        C = int(rng.integers(1, 300))
        psteps = int(rng.choice([4, 8, 16, 32]))
        DP = [int(v) for v in rng.integers(0, 2**63, C + 1, dtype=np.uint64)]
        EP = [int(v) for v in rng.integers(0, 2**63, C + 1, dtype=np.uint64)]
        for b in range(-(-2 * C // psteps)):
            x0 = pack_start(C, psteps, b, DP, EP)
            s0 = b * psteps
            assert max(0, s0 - C) <= x0 <= min(s0, C)
