"""Host model of the stream-K split of the gather kernel (gett.hip,
gett_sk_kernel and gett_fixup_kernel).

The last `tiles` output tiles are cut into BK-step pieces shared equally by
`blocks` workgroups; a piece that is a whole tile is written directly, the
others go to workspace slot 2*s (the workgroup's first tile) or 2*s + 1 (its
last tile) and are summed per tile, in workgroup order, by the fixup kernel.
This mirror re-derives every piece and checks that the steps of every tile
are covered exactly once, that every slot index lies inside the 2*blocks
slots the plan allocates, that no slot is written twice, and that the fixup
reads exactly the slots written for its tile.  The same for the balanced
schedule's pieces (gett_whole_piece_kernel, gett_piece_fixup_kernel).  The mirror
must be kept in step with the device code.
"""
import pytest


def sk_begin(I, S, s):
    return I * s // S


def sk_owner(I, S, x):
    s = min(x * S // I, S - 1)
    while s + 1 < S and sk_begin(I, S, s + 1) <= x:
        s += 1
    while s > 0 and sk_begin(I, S, s) > x:
        s -= 1
    return s


def pieces(tiles, blocks, nk):
    """(block, tile, k_begin, k_end, slot or None) of every piece."""
    I = tiles * nk
    out = []
    for s in range(blocks):
        a, b = sk_begin(I, blocks, s), sk_begin(I, blocks, s + 1)
        it = a
        while it < b:
            tt = it // nk
            ks = it - tt * nk
            ke = min(ks + (b - it), nk)
            whole = ks == 0 and ke == nk
            slot = None if whole else 2 * s + (0 if tt == a // nk else 1)
            out.append((s, tt, ks, ke, slot))
            it += ke - ks
    return out


def fixup_reads(tiles, blocks, nk, tt):
    I = tiles * nk
    lo, hi = sk_owner(I, blocks, tt * nk), sk_owner(I, blocks, (tt + 1) * nk - 1)
    if lo == hi:
        return None
    return [2 * s + (0 if tt == sk_begin(I, blocks, s) // nk else 1) for s in range(lo, hi + 1)
            if sk_begin(I, blocks, s) != sk_begin(I, blocks, s + 1)]


CASES = [(64, 512, 192), (64, 512, 96), (1, 7, 5), (3, 2, 10), (5, 5, 1), (7, 3, 4), (10, 64, 8), (13, 8, 100),
         (2, 16, 3), (4, 1, 9), (100, 256, 2), (1, 1, 1), (33, 50, 7)]


@pytest.mark.parametrize("tiles,blocks,nk", CASES)
def test_pieces_cover_every_step_once(tiles, blocks, nk):
    cover = {}
    for s, tt, ks, ke, slot in pieces(tiles, blocks, nk):
        assert 0 <= tt < tiles and 0 <= ks < ke <= nk
        for k in range(ks, ke):
            assert (tt, k) not in cover
            cover[(tt, k)] = s
    assert len(cover) == tiles * nk


@pytest.mark.parametrize("tiles,blocks,nk", CASES)
def test_slots_in_range_and_unique(tiles, blocks, nk):
    seen = set()
    for s, tt, ks, ke, slot in pieces(tiles, blocks, nk):
        if slot is None:
            continue
        assert 0 <= slot < 2 * blocks
        assert slot not in seen
        seen.add(slot)


@pytest.mark.parametrize("tiles,blocks,nk", CASES)
def test_fixup_reads_what_was_written(tiles, blocks, nk):
    by_tile = {}
    for s, tt, ks, ke, slot in pieces(tiles, blocks, nk):
        by_tile.setdefault(tt, []).append((s, ks, ke, slot))
    for tt in range(tiles):
        ps = sorted(by_tile[tt])
        reads = fixup_reads(tiles, blocks, nk, tt)
        if len(ps) == 1:
            # one workgroup held the whole tile and wrote C itself
            assert reads is None and ps[0][3] is None
        else:
            assert reads == [p[3] for p in ps]          # workgroup order = summation order
            assert all(p[3] is not None for p in ps)


def test_owner_matches_shares():
    for tiles, blocks, nk in CASES:
        I = tiles * nk
        for x in range(0, I, max(1, I // 200)):
            s = sk_owner(I, blocks, x)
            assert sk_begin(I, blocks, s) <= x < sk_begin(I, blocks, s + 1)


# ---- the balanced schedule (gett_whole_piece_kernel, gett_piece_fixup_kernel) ----
# S workgroups share R leftover tiles: tile r takes workgroups
# first(r) = floor(S r / R) .. first(r + 1) - 1, workgroup b finds its tile as
# r = floor(((b + 1) R - 1) / S) and its piece j = b - first(r) of P = first(r
# + 1) - first(r) pieces covers the summation indices
# [floor(nk j / P) BK, floor(nk (j + 1) / P) BK) clipped to K.

def even_first(S, R, r):
    return S * r // R


def even_pieces(S, R, K, BK):
    nk = -(-K // BK)
    out = []
    for b in range(S):
        r = ((b + 1) * R - 1) // S
        f0 = even_first(S, R, r)
        P = even_first(S, R, r + 1) - f0
        j = b - f0
        k0 = nk * j // P * BK
        k1 = nk * (j + 1) // P * BK
        out.append((b, r, k0, min(k1, K) - k0, P))
    return out


@pytest.mark.parametrize("S,R", [(512, 64), (512, 73), (512, 253), (512, 256), (1024, 216), (768, 240),
                                 (256, 1), (7, 3), (5, 2), (2048, 824)])
@pytest.mark.parametrize("K", [3072, 232, 16 * 35 - 8])
def test_balanced_pieces_cover_each_leftover_tile_once(S, R, K):
    BK = 16
    nk = -(-K // BK)
    P_max = -(-S // R)
    if nk < 4 * P_max:
        pytest.skip("the planner needs at least four steps per piece")
    ps = even_pieces(S, R, K, BK)
    # every workgroup has one piece; the owner formula inverts first()
    for b, r, k0, kn, P in ps:
        assert 0 <= r < R
        assert even_first(S, R, r) <= b < even_first(S, R, r + 1)
        assert P >= 2 and kn > 0
        # the piece kernel's summation range lies inside the tables
        assert 0 <= k0 and k0 + kn <= K
    # per tile: pieces in slot order tile [0, K) without gaps or overlaps
    for r in range(R):
        mine = [(k0, kn) for b, rr, k0, kn, P in ps if rr == r]
        assert len(mine) == even_first(S, R, r + 1) - even_first(S, R, r)
        at = 0
        for k0, kn in mine:
            assert k0 == at
            at += kn
        assert at == K
        # piece lengths differ by at most one step within a tile
        lens = [kn for k0, kn in mine[:-1]]
        if lens:
            assert max(lens) - min(lens) <= BK
    # piece counts differ by at most one between tiles
    counts = [even_first(S, R, r + 1) - even_first(S, R, r) for r in range(R)]
    assert max(counts) - min(counts) <= 1
