"""The autotuner's candidate lists (host logic, no GPU): every setting it
would time is one the knobs accept, and the tiled variants it is meant to
compare are present."""

import pytest

from paper_1104_0737_amd import autotune, binding as B


def _valid(setting, L, prec):
    s = autotune._full(setting)
    g, t, sp, pr, nt, ch, tile, once, lg = s
    assert len(setting) <= 9
    assert L % g == 0 and t in (64, 128, 192, 256) and sp in (0, 2, 4) and pr in (0, 1) and nt in (0, 1)
    assert 0 <= ch <= 4 and (ch == 0 or L % ch == 0)
    assert tile in (0, 1, 2, 3) and once in (0, 1)
    assert not (tile == 2 and prec == B.FP16S)      # the folded update is withdrawn for FP16 storage
    assert lg == 0 or (L % lg == 0 and tile in (1, 2, 3))


@pytest.mark.parametrize("prec", [B.FP64, B.FP32, B.FP16S])
@pytest.mark.parametrize("L", [12, 5])
def test_candidates_valid(prec, L):
    ops = autotune.operator_candidates(L, prec)
    for s in ops:
        _valid(s, L, prec)
    assert len(set(map(autotune._full, ops))) == len(ops)
    # pretend the first tiled setting was fastest
    times = {s: 1.0 for s in ops}
    times[next(s for s in ops if autotune._tiled(s))] = 0.5
    cands = autotune.sap_candidates(L, prec, times)
    for s in cands:
        _valid(s, L, prec)
    full = set(map(autotune._full, cands))
    # tiled with whole- and half-LDS tiles, and (even L) half the columns per workgroup, psi formed once or not
    for tile in (1, 3):
        for once in (0, 1):
            assert any(f[6] == tile and f[7] == once and f[8] == 0 for f in full), (tile, once)
            if L % 4 == 0 or (prec == B.FP64 and L % 2 == 0):
                assert any(f[6] == tile and f[7] == once and f[8] == L // 2 for f in full), (tile, once)
    assert any(f[6] == 2 for f in full) == (prec != B.FP16S)
