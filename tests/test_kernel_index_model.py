"""Host model of the GETT loader's index arithmetic (gett.hip, struct Loader).

The kernel gathers operand tiles through offset tables and, to keep its loop
free of branches, also loads past the last summation step from clamped
indices and masks the values afterwards.  This test re-derives, for every
loader variant (K- or row-contiguous, vector or element loads) and for
ragged and full-size extents, every (row, k) index pair the kernel touches
and every table entry it reads, and checks that all of them lie inside the
tensor -- and that every 16-byte vector stays inside one contiguous run.
The mirror must be kept in step with the device code.
"""
import numpy as np
import pytest

NT = 256


def loader_indices(R, BK, VEC, layout, vec, Rtot, K, NT=256):
    """Sets of accessed rows, k indices and vector starts of one operand."""
    P = R * BK // (VEC * NT)
    assert P >= 1 and P * VEC * NT == R * BK
    ids = np.arange(NT)[:, None] + NT * np.arange(P)[None, :]
    assert ids.max() < R * BK // VEC
    if layout == 0:
        rr = ids // (BK // VEC)
        kk = (ids % (BK // VEC)) * VEC
    else:
        kk = ids // (R // VEC)
        rr = (ids % (R // VEC)) * VEC
    rows, ks, vec_rows, vec_ks, tab_r, tab_k = [], [], [], [], [], []
    ntiles = (Rtot + R - 1) // R
    for t in range(ntiles):
        gr = t * R + rr
        for i in range(VEC):
            g = gr if (layout == 0 or vec) else gr + i
            used = np.where(g < Rtot, g, 0)            # roff[p][i] = offR[ok ? g : 0]
            tab_r.append(used.ravel())
            if layout == 0:
                if i == 0:
                    rows.append(used.ravel())            # K-contiguous: one row per vector
            else:
                if vec:
                    if i == 0:
                        vec_rows.append(used.ravel())   # the vector covers used .. used+VEC-1
                else:
                    rows.append(used.ravel())
    nsteps = (K + BK - 1) // BK
    last = K - VEC if (layout == 0 and vec) else K - 1
    # fetch_k is called for steps 0 .. nsteps + 1, load for 0 .. nsteps
    for s in range(nsteps + 2):
        k = s * BK + kk
        nko = VEC if layout == 0 else 1
        for i in range(nko):
            ki = k + (i if (layout == 0 and not vec) else 0)
            kc = np.where(ki <= last, ki, last)
            tab_k.append(kc.ravel())
            if s <= nsteps:
                if layout == 0 and vec:
                    if i == 0:
                        vec_ks.append(kc.ravel())
                else:
                    ks.append(kc.ravel())
    cat = lambda xs: np.concatenate(xs) if xs else np.zeros(0, dtype=np.int64)
    return cat(rows), cat(ks), cat(vec_rows), cat(vec_ks), cat(tab_r), cat(tab_k)


# (BM, BN, BK, waves) of the kernel's tile table
TILES = [(128, 128, 16, 4), (64, 64, 16, 4), (128, 128, 32, 4), (128, 128, 16, 8), (256, 128, 16, 8),
         (128, 64, 16, 4), (64, 128, 16, 4), (96, 96, 16, 4), (128, 96, 32, 8), (192, 96, 32, 8)]


@pytest.mark.parametrize("VEC", [2, 4])
@pytest.mark.parametrize("layout", [0, 1])
@pytest.mark.parametrize("vec", [True, False])
@pytest.mark.parametrize("R,BK,NTl", sorted({(t[0], t[2], 64 * t[3]) for t in TILES} |
                                             {(t[1], t[2], 64 * t[3]) for t in TILES}))
@pytest.mark.parametrize("Rtot,K", [(3072, 3072), (8192, 32), (16384, 32), (480, 480), (13, 7), (1, 1),
                                    (96, 30), (250, 12), (4, 4), (17, 8)])
def test_every_access_in_range(VEC, layout, vec, R, BK, NTl, Rtot, K):
    # vector loads are only planned when the contiguous dimension is a multiple of VEC
    if vec and ((layout == 0 and K % VEC) or (layout == 1 and Rtot % VEC)):
        pytest.skip("vector mode not planned for this extent")
    if R * BK % (VEC * NTl):
        pytest.skip("tile does not split for this vector width")
    rows, ks, vrows, vks, tr, tk = loader_indices(R, BK, VEC, layout, vec, Rtot, K, NTl)
    assert tr.min() >= 0 and tr.max() < Rtot, "row-table index out of range"
    assert tk.min() >= 0 and tk.max() < K, "k-table index out of range"
    if rows.size:
        assert rows.max() < Rtot and rows.min() >= 0
    if ks.size:
        assert ks.max() < K and ks.min() >= 0
    if vrows.size:
        assert np.all(vrows % VEC == 0) and (vrows + VEC - 1).max() < Rtot
    if vks.size:
        assert np.all(vks % VEC == 0) and (vks + VEC - 1).max() < K


def test_model_catches_the_unaligned_clamp():
    """The clamp to K-1 (instead of K-VEC) for K-contiguous vectors reads
    past the tensor; the model must flag it."""
    R, BK, VEC, Rtot, K = 128, 16, 2, 3072, 3072
    P = R * BK // (VEC * NT)
    ids = np.arange(NT)[:, None] + NT * np.arange(P)[None, :]
    kk = (ids % (BK // VEC)) * VEC
    nsteps = (K + BK - 1) // BK
    k = nsteps * BK + kk
    bad = np.where(k <= K - 1, k, K - 1)
    assert (bad + VEC - 1).max() >= K


# (BM, BN, BK, WGM, WGN) of the kernel's tile table, for the LDS check below
TILE_WAVES = [(128, 128, 16, 2, 2), (64, 64, 16, 2, 2), (128, 128, 32, 2, 2), (128, 128, 16, 4, 2),
              (256, 128, 16, 4, 2), (128, 64, 16, 2, 2), (64, 128, 16, 2, 2), (96, 96, 16, 2, 2),
              (128, 96, 32, 4, 2), (192, 96, 32, 4, 2)]


def test_tile_tables_agree():
    assert [(t[0], t[1], t[2], t[3] * t[4]) for t in TILE_WAVES] == TILES


@pytest.mark.parametrize("tile", range(len(TILE_WAVES)))
@pytest.mark.parametrize("tc_bytes,VEC", [(8, 2), (4, 4), (4, 2)])
@pytest.mark.parametrize("layoutA,layoutB", [(0, 0), (0, 1), (1, 0), (1, 1)])
def test_lds_positions_in_buffer(tile, tc_bytes, VEC, layoutA, layoutB):
    """Every LDS element a loader stores and every MFMA fragment read lies
    inside its operand's buffer (ELEMS = R * (BK + KPAD) for K-contiguous
    tiles, BK * (R + 4) otherwise), for every tile, layout and type pair."""
    BM, BN, BK, WGM, WGN = TILE_WAVES[tile]
    NTl = 64 * WGM * WGN
    KPAD = 2 if tc_bytes == 8 else 4
    for R, layout, W, wpos in ((BM, layoutA, BM // WGM, lambda w: (w // WGN)),
                               (BN, layoutB, BN // WGN, lambda w: (w % WGN))):
        if R * BK % (VEC * NTl):
            continue
        P = R * BK // (VEC * NTl)
        LDK, LDR = BK + KPAD, R + 4
        elems = R * LDK if layout == 0 else BK * LDR
        idx = (lambda r, k: r * LDK + k) if layout == 0 else (lambda r, k: k * LDR + r)
        ids = np.arange(NTl)[:, None] + NTl * np.arange(P)[None, :]
        if layout == 0:
            rr, kk = ids // (BK // VEC), (ids % (BK // VEC)) * VEC
            last = idx(rr, kk + VEC - 1)
        else:
            kk, rr = ids // (R // VEC), (ids % (R // VEC)) * VEC
            last = idx(rr + VEC - 1, kk)
        assert last.max() < elems and idx(rr, kk).min() >= 0
        # the stores of one pass cover the buffer's R x BK entries exactly once
        cover = set()
        for i in range(VEC):
            pos = idx(rr + (i if layout == 1 else 0), kk + (i if layout == 0 else 0))
            cover.update(pos.ravel().tolist())
        assert len(cover) == R * BK
        lane = np.arange(64)
        reads = []
        for w in range(WGM * WGN):
            r0 = wpos(w) * W
            for f in range(W // 16):
                for k4 in range(0, BK, 4):
                    reads.append(idx(r0 + f * 16 + (lane & 15), k4 + (lane >> 4)))
        reads = np.concatenate(reads)
        assert reads.min() >= 0 and reads.max() < elems
        assert set(reads.tolist()) <= cover


# ---- the short-summation kernel's staging schedule (gett.hip, gett_shortk_kernel)
def shortk_schedule(ntile):
    """Replay the LDS staging of one workgroup with `ntile` tiles: which tile's
    row offsets and C offsets each parity buffer holds when it is read, and
    which operand buffer holds which tile when it is multiplied.  Returns the
    list of (step, buffer, tile read, tile expected) for every read."""
    clamp = lambda j: min(j, ntile - 1)
    rows = [None, None]   # tile whose row offsets each buffer holds
    ctab = [None, None]   # tile whose C offsets each buffer holds
    ops = [None, None]    # tile whose operands each LDS buffer holds
    reads = []
    # prologue: rows of tile 0 -> rows[0]; rows of tile 1 -> rows[1], C of tile 0 -> ctab[0]
    rows[0] = clamp(0)
    ctab[0] = clamp(0)
    rows[1] = clamp(1)
    ctab[0] = clamp(0)
    ops[0] = 0
    for j in range(ntile):
        jn = j + 1 if j + 1 < ntile else j
        reads.append(("rows", jn & 1, rows[jn & 1], jn))          # step 2: init_from the next tile's rows
        loaded = jn
        fetched_rows, fetched_c = clamp(j + 2), clamp(j + 1)
        reads.append(("mma", j & 1, ops[j & 1], j))               # step 3: products of tile j
        ops[(j + 1) & 1] = loaded                                 # step 4
        rows[j & 1] = fetched_rows
        ctab[(j + 1) & 1] = fetched_c
        reads.append(("ctab", j & 1, ctab[j & 1], j))             # step 5: stores of tile j
    return reads


@pytest.mark.parametrize("ntile", [1, 2, 3, 4, 5, 32])
def test_shortk_staging_reads_what_was_written(ntile):
    for what, buf, got, want in shortk_schedule(ntile):
        assert got is not None, (what, buf, "read before written")
        assert got == want, (what, buf, got, want)


def test_shortk_staging_without_the_prologue_row_copy_reads_unwritten_lds():
    """Regression for a fault: without staging tile 0's rows into rows[0] in
    the prologue, a workgroup with a single tile reloads its tile from an
    LDS buffer that nothing wrote (garbage row offsets)."""
    rows = [None, 1]      # only the prologue's rows of tile 1
    ntile = 1
    jn = 0
    assert rows[jn & 1] is None


# ---- the slicer's tile walk (split.hip: tile_pos, row_offsets, load_tile) ----
# A 64 x 64 tile, 256 threads, 16 elements each; V consecutive elements along
# the operand's unit-stride dimension form one vector load (V = 1: element
# loads).  Mirror of the device mapping, checked for full coverage, vector
# contiguity and in-range clamped addresses.

SPR, SPK, SPT = 64, 64, 256
SPI = SPR * SPK // SPT


def slicer_pos(layout, V, tid, e):
    if layout == 0:
        return tid // (SPK // V) + (SPT // (SPK // V)) * (e // V), (tid % (SPK // V)) * V + e % V
    return (tid % (SPR // V)) * V + e % V, tid // (SPR // V) + (SPT // (SPR // V)) * (e // V)


@pytest.mark.parametrize("layout", [0, 1])
@pytest.mark.parametrize("V", [1, 2, 4])
def test_slicer_tile_walk_covers_the_tile_once(layout, V):
    seen = {}
    for tid in range(SPT):
        for e in range(SPI):
            seen.setdefault(slicer_pos(layout, V, tid, e), []).append((tid, e))
    assert len(seen) == SPR * SPK and all(len(v) == 1 for v in seen.values())
    # a vector's V elements: consecutive along the unit-stride dimension,
    # starting at a multiple of V
    for tid in range(SPT):
        for e in range(0, SPI, V):
            r0, k0 = slicer_pos(layout, V, tid, e)
            for i in range(V):
                r, k = slicer_pos(layout, V, tid, e + i)
                if layout == 0:
                    assert (r, k) == (r0, k0 + i) and k0 % V == 0
                else:
                    assert (r, k) == (r0 + i, k0) and r0 % V == 0


@pytest.mark.parametrize("layout", [0, 1])
@pytest.mark.parametrize("V,R,K", [(1, 70, 37), (2, 70, 38), (2, 64, 130), (4, 68, 36), (4, 132, 64)])
def test_slicer_vector_loads_stay_inside_the_operand(layout, V, R, K):
    """Every (clamped) vector start lies inside the operand with its whole
    vector; elements masked out are exactly those outside it."""
    for r0 in range(0, R + SPR - 1, SPR):
        for k0 in range(0, K + SPK - 1, SPK):
            for tid in range(SPT):
                for e in range(0, SPI, V):
                    rl, kl = slicer_pos(layout, V, tid, e)
                    rlast = R - V if (layout == 1 and V > 1) else R - 1
                    klast = K - V if (layout == 0 and V > 1) else K - 1
                    r = min(r0 + rl, rlast)
                    k = min(k0 + kl, klast)
                    if layout == 0:
                        assert 0 <= r < R and 0 <= k and k + V <= K
                    else:
                        assert 0 <= k < K and 0 <= r and r + V <= R
                    # with the vectorized extent a multiple of V, a vector is
                    # wholly inside the operand or wholly outside (masked)
                    inside = [r0 + slicer_pos(layout, V, tid, e + i)[0] < R and
                              k0 + slicer_pos(layout, V, tid, e + i)[1] < K for i in range(V)]
                    assert all(inside) or not any(inside)
