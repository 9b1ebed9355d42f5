"""CPU model of the index maps of the 16384-point FFT in csrc/tfx_fft16k.hip.

The kernel's transform is 16384 = 16 x 16 x 16 x 4 over 1024 virtual lanes
of 16 values, with three exchanges through one LDS plane.  This model runs
the same passes in FP64 on the CPU with the kernel's address maps written
out again here, and checks that
  - every exchange's write and read maps are bijections onto [0, 16384),
  - the forward composition equals the DFT (numpy's FFT) and the inverse
    composition undoes it (times 16384),
  - every access of a wave (64 consecutive virtual lanes, one value index) is
    free of LDS bank conflicts: 64 distinct banks for 4-byte accesses, and for
    the 16-byte group accesses of pass D each quarter-wave covers the 64 banks
    once.
"""
import numpy as np
import pytest

NB = 16384
LANES = 1024


def coords(L):
    return dict(L=L, k1=L >> 6, c=L & 63, d=(L & 63) >> 2, e=L & 3, k2=(L >> 2) & 15, q=L & 3)


def rot(base, step, r, j):
    return base + step * j - (64 if j >= 16 - r else 0)


def map_a(l, j):
    return 1024 * j + l["L"]


def map_b(l, j):
    return 1024 * l["k1"] + 64 * j + l["c"]


def rot_w(l, j):
    return rot(1024 * l["k1"] + 4 * l["d"] + l["e"], 68, l["d"], j)


def rot_c(l, j):
    return rot(1024 * l["k1"] + 68 * l["k2"] + l["e"], 4, l["k2"], j)


def group_addr(l, r):
    return 1024 * l["k1"] + 64 * l["k2"] + 4 * ((4 * l["q"] + r + l["k2"]) & 15)


LANE = [coords(L) for L in range(LANES)]


def dft(v, sign):
    n = len(v)
    k = np.arange(n)
    return np.exp(sign * 2j * np.pi * np.outer(k, k) / n) @ v


def exchange(val, wmap, rmap):
    P = np.full(NB, np.nan + 0j)
    for L in range(LANES):
        for j in range(16):
            P[wmap(LANE[L], j)] = val[L, j]
    out = np.empty_like(val)
    for L in range(LANES):
        for j in range(16):
            out[L, j] = P[rmap(LANE[L], j)]
    return out


def to_groups(val):
    P = np.full(NB, np.nan + 0j)
    for L in range(LANES):
        for j in range(16):
            P[rot_c(LANE[L], j)] = val[L, j]
    out = np.empty_like(val)
    for L in range(LANES):
        for r in range(4):
            a = group_addr(LANE[L], r)
            out[L, 4 * r:4 * r + 4] = P[a:a + 4]
    return out


def from_groups(val):
    P = np.full(NB, np.nan + 0j)
    for L in range(LANES):
        for r in range(4):
            a = group_addr(LANE[L], r)
            P[a:a + 4] = val[L, 4 * r:4 * r + 4]
    out = np.empty_like(val)
    for L in range(LANES):
        for j in range(16):
            out[L, j] = P[rot_c(LANE[L], j)]
    return out


def twiddle(val, which, conj):
    out = val.copy()
    for L in range(LANES):
        l = LANE[L]
        m = {"A": l["L"], "B": 16 * l["c"], "C": 256 * l["e"]}[which]
        w = np.exp(-2j * np.pi * ((m * np.arange(16)) % NB) / NB)
        out[L] *= np.conj(w) if conj else w
    return out


def forward(z):
    """Input: lane L holds z[1024 a + L] at a.  Output in pass D's layout."""
    v = np.stack([z[np.arange(16) * 1024 + L] for L in range(LANES)])
    v = twiddle(np.stack([dft(r, -1) for r in v]), "A", False)
    v = exchange(v, map_a, map_b)
    v = twiddle(np.stack([dft(r, -1) for r in v]), "B", False)
    v = exchange(v, rot_w, rot_c)
    v = twiddle(np.stack([dft(r, -1) for r in v]), "C", False)
    v = to_groups(v)
    return np.stack([np.concatenate([dft(r[4 * g:4 * g + 4], -1) for g in range(4)]) for r in v])


def inverse(v):
    v = np.stack([np.concatenate([dft(r[4 * g:4 * g + 4], 1) for g in range(4)]) for r in v])
    v = from_groups(v)
    v = np.stack([dft(r, 1) for r in twiddle(v, "C", True)])
    v = exchange(v, rot_c, rot_w)
    v = np.stack([dft(r, 1) for r in twiddle(v, "B", True)])
    v = exchange(v, map_b, map_a)
    v = np.stack([dft(r, 1) for r in twiddle(v, "A", True)])
    z = np.empty(NB, complex)
    for L in range(LANES):
        z[np.arange(16) * 1024 + L] = v[L]
    return z


def spectrum_index(L, j):
    l = LANE[L]
    r, k4 = j // 4, j % 4
    return l["k1"] + 16 * l["k2"] + 256 * (4 * l["q"] + r) + 4096 * k4


@pytest.mark.parametrize("wmap,rmap", [(map_a, map_b), (rot_w, rot_c), (rot_c, rot_w), (map_b, map_a)])
def test_exchange_maps_are_bijections(wmap, rmap):
    for m in (wmap, rmap):
        addrs = sorted(m(LANE[L], j) for L in range(LANES) for j in range(16))
        assert addrs == list(range(NB))


def test_group_map_is_a_bijection():
    addrs = sorted(group_addr(LANE[L], r) + i for L in range(LANES) for r in range(4) for i in range(4))
    assert addrs == list(range(NB))


def test_forward_is_the_dft_and_inverse_undoes_it():
    rng = np.random.default_rng(16384)
    z = rng.standard_normal(NB) + 1j * rng.standard_normal(NB)
    v = forward(z)
    ref = np.fft.fft(z)
    got = np.empty(NB, complex)
    for L in range(LANES):
        for j in range(16):
            got[spectrum_index(L, j)] = v[L, j]
    assert np.max(np.abs(got - ref)) <= 1e-12 * np.max(np.abs(ref))
    back = inverse(v) / NB
    assert np.max(np.abs(back - z)) <= 1e-12 * np.max(np.abs(z))


@pytest.mark.parametrize("m", [map_a, map_b, rot_w, rot_c])
def test_scalar_accesses_are_free_of_bank_conflicts(m):
    for w in range(LANES // 64):
        for j in range(16):
            banks = [m(LANE[64 * w + i], j) % 64 for i in range(64)]
            assert len(set(banks)) == 64, (m.__name__, w, j)
            for h in (0, 32):
                assert len(set(b % 32 for b in banks[h:h + 32])) == 32


def test_group_accesses_are_free_of_bank_conflicts():
    for w in range(LANES // 64):
        for r in range(4):
            for qw in range(4):
                banks = []
                for i in range(16):
                    a = group_addr(LANE[64 * w + 16 * qw + i], r)
                    banks += [(a + u) % 64 for u in range(4)]
                assert len(set(banks)) == 64, (w, r, qw)
