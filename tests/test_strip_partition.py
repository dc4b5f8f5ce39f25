"""Host model of the symmetric product's strip sweep (strip_product and
strip_gather in csrc/solve.hip, strips_before / strip_slots in
csrc/bc_internal.h), checked against a dense product on the CPU.

The model restates the sweep's index arithmetic lane by lane: row block B
(128 rows) swept from column 128 B in strips of 16 VEC columns, equal
contiguous strip ranges for the 16 G wavefronts of a system, lane l holding
VEC entries of rows l/16 + 4 k of each 32-row batch, the lane-permute
reduce-scatters of the row and column sums, segment slots h + B and the
gather's enumeration of segments and column sums.  It checks that every entry
of the diagonal blocks and above is read exactly once, that no slot or column
sum is written twice, that the gather finds exactly the wavefronts holding
strips of a block and reads only written slots, and that y = V x and x^T V x
come out right, so that a mistake in the
partition (a strip counted twice, a slot shared, a segment the gather does not
find) fails here without a GPU."""

import numpy as np
import pytest

KRB = 128
LANES = np.arange(64)


def strips_before(B, ld, sw):
    return B * (ld // sw) - (KRB // sw) * (B * (B - 1) // 2)


def wg_count(N):
    return max(1, min(256, (N + 79) // 80))


def xor_lane(v, m):
    """Value of lane l ^ m in every lane l (a lane permute)."""
    return v[LANES ^ m]


def row16_scatter8(v):
    """Lane l keeps the sum over its 16-lane group of value 4 b3 + 2 b2 + b1."""
    b3, b2, b1 = (LANES & 8) != 0, (LANES & 4) != 0, (LANES & 2) != 0
    a = [np.where(b3, v[j + 4], v[j]) + xor_lane(np.where(b3, v[j], v[j + 4]), 8) for j in range(4)]
    b = [np.where(b2, a[j + 2], a[j]) + xor_lane(np.where(b2, a[j], a[j + 2]), 7) for j in range(2)]
    c = np.where(b1, b[1], b[0]) + xor_lane(np.where(b1, b[0], b[1]), 3)
    return c + xor_lane(c, 1)


def col4_scatter(cs, vec):
    """Column sums over the lanes l, l^16, l^32, l^48."""
    b4, b5 = (LANES & 16) != 0, (LANES & 32) != 0
    if vec == 4:
        a = [np.where(b4, cs[j + 2], cs[j]) + xor_lane(np.where(b4, cs[j], cs[j + 2]), 16) for j in range(2)]
        return np.where(b5, a[1], a[0]) + xor_lane(np.where(b5, a[0], a[1]), 32)
    c = np.where(b4, cs[1], cs[0]) + xor_lane(np.where(b4, cs[0], cs[1]), 16)
    return c + xor_lane(c, 32)


def test_row_reduce_scatter():
    rng = np.random.default_rng(0)
    v = rng.standard_normal((8, 64))
    got = row16_scatter8(v)
    for l in range(64):
        k = 4 * ((l >> 3) & 1) + 2 * ((l >> 2) & 1) + ((l >> 1) & 1)
        grp = (l & ~15) + np.arange(16)
        assert got[l] == pytest.approx(v[k, grp].sum(), rel=1e-13)


def strip_product_model(A, x, vec):
    """y = A x and x^T A x by the strip sweep; A symmetric N x N."""
    N = A.shape[0]
    ld = (N + 63) // 64 * 64
    SW = 16 * vec
    NDIAG = KRB // SW
    nB = (N + KRB - 1) // KRB
    T = strips_before(nB, ld, SW)
    G = wg_count(N)
    GH = 16 * G
    nslots = GH + nB
    assert nslots == 16 * G + nB
    rpart = np.full((nslots, KRB), np.nan)
    cpart = np.full((nB, ld), np.nan)
    Vp = np.zeros((N, ld))
    Vp[:, :N] = A
    xp = np.zeros(ld)
    xp[:N] = x
    rq, cq = LANES >> 4, LANES & 15
    cover = np.zeros((N, ld), dtype=np.int64)
    delta = 0.0
    for hold in range(GH):
        u, u1 = T * hold // GH, T * (hold + 1) // GH
        if u >= u1:
            continue
        B = max(b for b in range(nB) if strips_before(b, ld, SW) <= u)
        SE = strips_before(B + 1, ld, SW)
        c = u - strips_before(B, ld, SW)
        acc = [np.zeros(64) for _ in range(4)]
        while True:
            cs = [np.zeros(64) for _ in range(vec)]
            col = KRB * B + SW * c + vec * cq
            assert (col + vec <= ld).all()
            xq = [xp[col + q] for q in range(vec)]
            for h in range(4):
                rows = [KRB * B + rq + 32 * h + 4 * k for k in range(8)]
                va = []
                for k in range(8):
                    ok = rows[k] < N
                    for q in range(vec):
                        np.add.at(cover, (rows[k][ok], (col + q)[ok]), 1)
                    va.append([np.where(ok, Vp[np.minimum(rows[k], N - 1), col + q], 0.0) for q in range(vec)])
                # x of the batch's rows (from LDS in the kernel); zero past N
                xb = [np.where(rows[k] < N, xp[np.minimum(rows[k], ld - 1)], 0.0) for k in range(8)]
                rp = [sum(va[k][q] * xq[q] for q in range(vec)) for k in range(8)]
                for k in range(8):
                    for q in range(vec):
                        cs[q] = cs[q] + va[k][q] * xb[k]
                a0 = acc[0] + row16_scatter8(rp)
                acc = [acc[1], acc[2], acc[3], a0]
            delta += (1.0 if c < NDIAG else 2.0) * sum(float((xq[q] * cs[q]).sum()) for q in range(vec))
            more, same = u + 1 < u1, u + 1 < SE
            s_ = col4_scatter(cs, vec)
            qsel = 2 * ((LANES >> 4) & 1) + ((LANES >> 5) & 1) if vec == 4 else (LANES >> 4) & 1
            if c >= NDIAG:
                for l in range(64):
                    if vec == 4 or l < 32:
                        cc = KRB * B + SW * c + vec * cq[l] + qsel[l]
                        assert np.isnan(cpart[B, cc]), "column sum written twice"
                        cpart[B, cc] = s_[l]
            if not more or not same:
                slot = hold + B
                assert slot < nslots
                rk = 4 * ((LANES >> 1) & 7) + rq
                for hh in range(4):
                    for l in range(0, 64, 2):
                        row = 32 * hh + rk[l]
                        if KRB * B + row < N:
                            assert np.isnan(rpart[slot, row]), "slot written twice"
                            rpart[slot, row] = acc[hh][l]
                acc = [np.zeros(64) for _ in range(4)]
            if not more:
                break
            u += 1
            if same:
                c += 1
            else:
                B, c = B + 1, 0
                SE = strips_before(B + 1, ld, SW)
    for i in range(N):
        Bi = i // KRB
        assert (cover[i, KRB * Bi:N] == 1).all() and (cover[i, :KRB * Bi] == 0).all(), i
    y = np.zeros(N)
    for i in range(N):
        B = i // KRB
        SB, SEb = strips_before(B, ld, SW), strips_before(B + 1, ld, SW)
        glo = ((SB + 1) * GH + T - 1) // T - 1
        ghi = (SEb * GH + T - 1) // T - 1
        for g in range(GH):
            lo, hi = T * g // GH, T * (g + 1) // GH
            holds = lo < hi and lo < SEb and hi > SB
            assert holds == (glo <= g <= ghi and T * (g + 1) // GH != T * g // GH), (i, g)
            if holds:
                v = rpart[g + B, i - KRB * B]
                assert not np.isnan(v), (i, g)
                y[i] += v
        for A_ in range(B):
            assert not np.isnan(cpart[A_, i])
            y[i] += cpart[A_, i]
    return y, delta


@pytest.mark.parametrize("N,vec", [(1, 4), (37, 4), (128, 2), (130, 4), (300, 2), (300, 4)])
def test_strip_sweep_model(N, vec):
    rng = np.random.default_rng(N + vec)
    A = rng.standard_normal((N, N))
    A = A + A.T
    x = rng.standard_normal(N)
    y, delta = strip_product_model(A, x, vec)
    scale = np.abs(A) @ np.abs(x)
    assert (np.abs(y - A @ x) <= 1e-12 * scale + 1e-300).all()
    assert delta == pytest.approx(float(x @ A @ x), rel=1e-10, abs=1e-10 * float(np.abs(x) @ np.abs(A) @ np.abs(x)))
