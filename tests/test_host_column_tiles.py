"""Host check of the class passes' column tiles (llr_sweep.hip: col_tile,
col_nbr, staples, col_staples, the sampler queue's counter): for every
lane of every tile, including lanes past the end of the (x0h, x1, x2) slab
and the x3 tail, every index the kernels load lies inside its plane, every
per-lane part of an index is a position in the slab, the links of valid
lanes are the class's links exactly once with the right neighbours, and a
queue entry's Philox word 0 is its link's half index.  (A lane past the
slab that loaded position 0 with the offsets of its own, out-of-range,
coordinates once read outside the state.)"""
import numpy as np
import pytest

kBlock = 256


def _half(y, L):
    return (y[0] % L + L * ((y[1] % L) + L * ((y[2] % L) + L * (y[3] % L)))) >> 1


@pytest.mark.parametrize("L", [2, 4, 6, 8, 10, 12, 20])
@pytest.mark.parametrize("LPT", [1, 2, 4])
@pytest.mark.parametrize("p", [0, 1])
def test_column_tile_addressing(L, LPT, p):
    hL, V2 = L // 2, L ** 4 // 2
    P = V2 // L
    npt = (P + kBlock - 1) // kBlock
    hstr = [0, hL, hL * L, hL * L * L]
    hwrap = [0] + [(L - 1) * hstr[d] for d in (1, 2, 3)]
    tid = np.arange(kBlock)
    seen = np.zeros(V2, dtype=np.int64)
    for tile in range(npt * ((L + LPT - 1) // LPT)):
        xg, pt = divmod(tile, npt)
        pos0 = pt * kBlock
        in_slab = pos0 + tid < P
        pos = np.where(in_slab, pos0 + tid, 0)                 # col_tile
        r1 = pos // hL
        x0h, x1, x2 = pos - r1 * hL, (r1 % L), r1 // L
        x3_0 = xg * LPT
        b0 = (p + x1 + x2 + x3_0) & 1                           # col_nbr
        uo = np.where(x0h == hL - 1, 1 - hL, 1)
        de = np.where(x0h == 0, hL - 1, -1)
        up0 = [np.where(b0 == 1, uo, 0), np.where(b0 == 1, 0, uo)]
        dn0 = [np.where(b0 == 1, 0, de), np.where(b0 == 1, de, 0)]
        up1, dn1 = np.where(x1 == L - 1, -hwrap[1], hstr[1]), np.where(x1 == 0, hwrap[1], -hstr[1])
        up2, dn2 = np.where(x2 == L - 1, -hwrap[2], hstr[2]), np.where(x2 == 0, hwrap[2], -hstr[2])
        for r in range(LPT):
            x3 = x3_0 + r
            valid = in_slab & (x3 < L)
            hl = pos + P * x3
            if x3 < L:                                          # staples
                K = r & 1
                vu, vd = [up0[K], up1, up2, 0], [dn0[K], dn1, dn2, 0]
                sh = P * x3
                su = [sh, sh, sh, sh + (-hwrap[3] if x3 == L - 1 else hstr[3])]
                sd = [0, 0, 0, hwrap[3] if x3 == 0 else -hstr[3]]
                x = [2 * x0h + ((p + x1 + x2 + x3) & 1), x1, x2, np.full(kBlock, x3)]
                for MU in range(4):
                    for NU in range(4):
                        if NU == MU:
                            continue
                        for uni, lane, shift in ((su[MU], vu[MU], (MU, +1, None)), (su[NU], vu[NU], (NU, +1, None)),
                                                 (sh, 0, None), (su[MU] + sd[NU], vu[MU] + vd[NU], (MU, +1, NU)),
                                                 (sh + sd[NU], vd[NU], (NU, -1, None))):
                            ln = pos + lane
                            assert np.all((ln >= 0) & (ln < P))
                            idx = ln + uni
                            assert np.all((idx >= 0) & (idx < V2))
                            if shift is not None:               # the neighbour it names
                                y = [c.copy() for c in x]
                                d, sgn, d2 = shift
                                y[d] = y[d] + sgn
                                if d2 is not None:
                                    y[d2] = y[d2] - 1
                                want = _half(y, L)
                                assert np.array_equal(idx[valid], want[valid])
                assert np.all(hl[valid] == _half(x, L)[valid])
                assert np.all((np.array(x)[:, valid].sum(0) & 1) == p)
            np.add.at(seen, hl[valid], 1)
            e = r * kBlock + tid                                # sampler queue entry
            he = pos0 + (e & (kBlock - 1)) + P * (x3_0 + e // kBlock)
            assert np.array_equal(he[valid], hl[valid])
    assert np.all(seen == 1)
