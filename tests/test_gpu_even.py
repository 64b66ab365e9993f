"""The balanced schedule of the gather kernel against the oracle: whole tiles
for the full rounds of resident workgroups, then the tiles left over cut into
one more full round of equal summation pieces (summed in piece order by a
fix-up kernel).  Ragged edges, both storage types, several tiles and operand
layouts, leftover tiles alone (no full round) and after one or two rounds,
piece counts that differ by one between tiles, beta 0 and beta != 0, and the
planner taking it for the CCSD-like contraction at its full size."""
import numpy as np
import pytest

from gpu_common import TOL, inputs, oracle, print_case, shape_of, to_np, torch_dev

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
comet = pytest.importorskip("paper_2102_06827_amd")

TILE_SHAPE = {0: (128, 128, 16), 1: (64, 64, 16), 3: (128, 128, 16)}


def cus():
    return torch.cuda.get_device_properties(0).multi_processor_count


def slots(tile, dtype, monkeypatch):
    """Resident workgroups of the whole-tile kernel of `tile` on the device."""
    monkeypatch.setenv("COMET_GETT_TILE", str(tile))
    A = torch.zeros((8, 8, 8, 8), dtype=dtype, device="cuda")
    B = torch.zeros((8, 8, 8, 8), dtype=dtype, device="cuda")
    return comet.Plan("abij=acik*bkcj", A, B, path="gett").describe()["resident"] * cus()


def shape_for(tile, S, rounds, frac):
    """Extents of abij=acik*bkcj (M = a*i, N = b*j, K = c*k) whose tile grid
    has `rounds` full rounds of S tiles plus about frac * S leftover tiles,
    with ragged M, N and K edges, vector-friendly runs (i = 12, j = k = 8)
    and a summation of at least four steps per piece."""
    bm, bn, bk = TILE_SHAPE[tile]
    want = rounds * S + max(1, int(frac * S))
    tn = max(2, int(np.sqrt(want / 3)))
    while True:
        tm = -(-want // tn)
        T = tm * tn
        R = T - (T // S) * S
        # the pieces' round holds at least half as many workgroups as a
        # round of whole tiles: at least two pieces per leftover tile
        if T // S == rounds and 0 < R and 4 * R <= S:
            break
        tn += 1
    P = -(-S // R)
    nk = 4 * P + 3
    a = (tm * bm - 1) // 12               # M = 12 a: last tile row ragged
    b = (tn * bn - 8) // 8                # N = 8 b: last tile column 8 short
    c = 2 * nk - 1                        # K = 8 c = 16 nk - 8: last step half full
    assert -(-12 * a // bm) == tm and -(-8 * b // bn) == tn
    return dict(a=a, i=12, b=b, j=8, c=c, k=8), T, R


CASES = [
    # tile, dtype, full rounds, leftover fraction of a round
    (3, torch.float64, 0, 0.19),
    (3, torch.float64, 1, 0.125),
    (3, torch.float64, 1, 0.24),
    (3, torch.float32, 1, 0.22),
    (1, torch.float64, 1, 0.21),
    (1, torch.float32, 2, 0.24),
    (0, torch.float64, 1, 0.2),
]


@pytest.mark.parametrize("tile,dtype,rounds,frac", CASES)
def test_balanced_schedule_matches_oracle(tile, dtype, rounds, frac, monkeypatch):
    S = slots(tile, dtype, monkeypatch)
    ext, T, R = shape_for(tile, S, rounds, frac)
    spec = "abij=acik*bkcj"
    monkeypatch.setenv("COMET_GETT_TILE", str(tile))
    monkeypatch.setenv("COMET_GETT_EVEN", "1")
    name = "f64" if dtype == torch.float64 else "f32"
    cast = np.float64 if dtype == torch.float64 else np.float32
    runs = [("integer", 1.0, 1.0, 8101), ("uniform", -0.75, 0.5, 8111)]
    if rounds == 1 and tile == 3:
        runs.append(("integer", 2.0, 0.0, 8121))
    for kind, alpha, beta, seed in runs:
        print_case("balanced", tile, name, rounds, frac, ext, kind, beta)
        A, B, C0 = inputs(spec, ext, seed + tile, kind=kind, beta=True)
        Ad, Bd, Cd = torch_dev(A, dtype), torch_dev(B, dtype), torch_dev(C0, dtype)
        plan = comet.Plan(spec, Ad, Bd, Cd, path="gett")
        d = plan.describe()
        assert d["tile"] == tile and d["even"] == 1, d
        # full rounds of S whole tiles; the pieces' round holds at most S
        assert d["even_whole"] == rounds * S and d["sk_tiles"] == R and 2 * R <= d["sk_blocks"] <= S
        assert plan.workspace_bytes >= d["sk_blocks"] * TILE_SHAPE[tile][0] * TILE_SHAPE[tile][1] * (
            8 if name == "f64" else 4)
        plan(Ad, Bd, Cd, alpha=alpha, beta=beta)
        torch.cuda.synchronize()
        ref = oracle.contract(spec, A.astype(cast), B.astype(cast), C0.astype(cast) if beta else None,
                              alpha=alpha, beta=beta)
        got = to_np(Cd)
        if kind == "integer":
            assert np.array_equal(got, ref), "integer inputs must match bit for bit"
        else:
            assert oracle.relerr(got, ref) <= TOL[name]


def test_balanced_schedule_is_deterministic(monkeypatch):
    """Pieces are summed in a fixed order: repeated runs agree bit for bit."""
    S = slots(3, torch.float64, monkeypatch)
    ext, _, _ = shape_for(3, S, 1, 0.25)
    spec = "abij=acik*bkcj"
    monkeypatch.setenv("COMET_GETT_EVEN", "1")
    A, B, _ = inputs(spec, ext, 8131, kind="uniform")
    Ad, Bd = torch_dev(A, torch.float64), torch_dev(B, torch.float64)
    plan = comet.Plan(spec, Ad, Bd, path="gett")
    assert plan.describe()["even"] == 1
    first = to_np(plan(Ad, Bd))
    for _ in range(3):
        assert np.array_equal(to_np(plan(Ad, Bd)), first)


def test_balanced_schedule_off_and_misaligned_operands(monkeypatch):
    """COMET_GETT_EVEN=0 keeps stream-K; a misaligned operand view runs whole
    tiles with the balanced plan's workspace -- both equal to the oracle."""
    S = slots(3, torch.float64, monkeypatch)
    ext, _, _ = shape_for(3, S, 1, 0.25)
    spec = "abij=acik*bkcj"
    c, a, b = oracle.split_spec(spec)
    A, B, _ = inputs(spec, ext, 8141, kind="integer")
    ref = oracle.contract(spec, A, B)
    monkeypatch.setenv("COMET_GETT_EVEN", "0")
    Ad, Bd = torch_dev(A, torch.float64), torch_dev(B, torch.float64)
    plan = comet.Plan(spec, Ad, Bd, path="gett")
    assert plan.describe()["even"] == 0
    assert np.array_equal(to_np(plan(Ad, Bd)), ref)
    monkeypatch.setenv("COMET_GETT_EVEN", "1")
    plan = comet.Plan(spec, Ad, Bd, path="gett")
    assert plan.describe()["even"] == 1
    # the same values one element into a larger buffer: 8-byte aligned only
    buf = torch.empty(Ad.numel() + 1, dtype=torch.float64, device="cuda")
    Am = buf[1:].view(Ad.shape)
    Am.copy_(Ad)
    print_case("balanced misaligned")
    assert np.array_equal(to_np(plan(Am, Bd)), ref)


def test_planner_takes_balanced_schedule_for_ccsd_contraction():
    """The CCSD-like contraction at full size (M = N = K = 3072, 576 tiles of
    128 x 128): whole tiles for the first full round, the rest as pieces;
    sampled outputs against the oracle, integer inputs bit for bit."""
    spec = "abij=acik*bkcj"
    V, O = 96, 32
    ext = dict(a=V, b=V, c=V, i=O, j=O, k=O)
    A, B, C0 = inputs(spec, ext, 8151, kind="integer", beta=True)
    print_case("balanced ccsd full")
    Ad, Bd, Cd = torch_dev(A, torch.float64), torch_dev(B, torch.float64), torch_dev(C0, torch.float64)
    plan = comet.Plan(spec, Ad, Bd, Cd)
    d = plan.describe()
    if d["tile"] == 3 and d["resident"] * cus() == 512:
        assert d["even"] == 1 and d["sk_tiles"] == 64 and d["sk_blocks"] == 512 and d["even_whole"] == 512
    plan(Ad, Bd, Cd, alpha=1.0, beta=-1.0)
    torch.cuda.synchronize()
    rng = np.random.default_rng(8152)
    shp = shape_of("abij", ext)
    pts = np.stack([rng.integers(0, e, 20000) for e in shp], axis=1)
    pts = np.concatenate([pts, np.zeros((1, 4), np.int64), np.array([shp]) - 1])
    idx = torch.from_numpy(pts).cuda()
    got = Cd[tuple(idx.T)].cpu().numpy()
    ref = oracle.contract_points(spec, A, B, pts, C0, 1.0, -1.0)
    assert np.array_equal(got, ref)
