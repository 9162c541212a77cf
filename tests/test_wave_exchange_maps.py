"""Host check of the in-wave exchange layouts of the N = 4096 radix-8 kernel.

The kernel (csrc/wavex.hpp) runs the Stockham passes of Section II-B with a
butterfly-to-lane map that changes per pass, so that the exchanges after
passes 0 and 2 become 8 x 8 transposes between lane bits and register legs
(v_permlane32_swap, v_permlane16_swap, a DPP row rotation by 8), and only the
exchange after pass 1 goes through a swizzled LDS buffer.  This test emulates
those maps and instructions lane by lane in numpy (complex128, numpy's DFT
matrices and FFT as the reference) for the three layouts the library
compiles, and checks:
  - the result is the DFT of Section II-A in both directions;
  - every LDS slot is written exactly once and read after it was written;
  - every access of 32 consecutive lanes hits 32 distinct 8-byte slots
    modulo 32 (all 64 four-byte banks once);
  - every global access stays inside its row.
The GPU parity tests run the compiled kernels against the oracle.
"""
import numpy as np
import pytest

N = 4096


def dft8_rows(v, inv):
    k = np.arange(8)
    m = np.exp((1 if inv else -1) * 2j * np.pi * np.outer(k, k) / 8)
    return v @ m.T


def twiddle(ns, k, r, inv):
    length = ns * 8
    w = np.exp(-2j * np.pi * ((k * r) % length) / length)
    return np.conj(w) if inv else w


def slot_one_member(i):
    q = i >> 6
    return i ^ (q & 7) ^ (((q ^ (q >> 3)) & 1) << 3) ^ (((q >> 1) & 1) << 4)


def slot_two_members(i):
    q = i >> 6
    return i ^ ((q >> 3) & 1) ^ ((q & 7) << 1) ^ ((((q >> 3) ^ q) & 1) << 4)


def cross_lane(p, q, bit, lanes):
    """(lane, p) and (lane ^ 2^bit, q) exchange where lane bit `bit` is 1 for
    p's lane: the permlane swaps for bits 4 and 5, DPP + select for bit 3."""
    lane = lanes & 63
    base = lanes - lane
    hi = ((lane >> bit) & 1) == 1
    partner = base + (lane ^ (1 << bit))
    return np.where(hi, q[partner], p), np.where(hi, q, p[partner])


def transpose(a, members, lanes):
    """a[s][r]: member bit k <-> leg bit k; member bits in the lane are lane
    bits 6 - LB + k, the others pick the lane's butterfly s."""
    lb = 3 if members == 1 else 2
    a = [[a[s][r].copy() for r in range(8)] for s in range(members)]
    for k in range(3):
        if k < lb:
            for s in range(members):
                for r in range(8):
                    if not (r >> k) & 1:
                        a[s][r], a[s][r | 1 << k] = cross_lane(a[s][r], a[s][r | 1 << k], 6 - lb + k, lanes)
        else:
            for r in range(4):
                a[1][r], a[0][r + 4] = a[0][r + 4], a[1][r]
    return a


def emulate(x, groups, members, inv):
    lb = 3 if members == 1 else 2
    gpw, ms = 64 >> lb, 1 << lb
    slot = slot_one_member if members == 1 else slot_two_members
    lanes = np.arange(512 // (groups * members))
    m0 = (lanes & 63) >> (6 - lb)
    g0 = groups * (gpw * (lanes >> 6) + (lanes & (gpw - 1)))
    accesses = []
    a = []
    for u in range(groups):
        au = []
        for s in range(members):
            pos = [g0 + u + 64 * (m0 + ms * s) + 512 * r for r in range(8)]
            assert all(p.min() >= 0 and p.max() < N for p in pos)
            au.append([x[p] for p in pos])
        a.append(au)

    def dfts(au):
        return [list(dft8_rows(np.stack(v, 1), inv).T) for v in au]

    for u in range(groups):
        a[u] = transpose(dfts(a[u]), members, lanes)
        for s in range(members):
            for r in range(1, 8):
                a[u][s][r] = a[u][s][r] * twiddle(8, m0 + ms * s, r, inv)
        a[u] = dfts(a[u])
    lds = np.full(N, np.nan + 0j)
    written = np.zeros(N, int)
    for u in range(groups):
        for s in range(members):
            base = 64 * (g0 + u) + m0 + ms * s
            sb = slot(base)
            for r in range(8):
                assert np.array_equal(sb ^ (8 * r), slot(base + 8 * r))
                lds[sb ^ (8 * r)] = a[u][s][r]
                written[sb ^ (8 * r)] += 1
                accesses.append(sb ^ (8 * r))
    assert np.all(written == 1)
    for u in range(groups):
        for s in range(members):
            base = g0 + u + 64 * (m0 + ms * s)
            s0, s1 = slot(base), slot(base + 512)
            for r in range(8):
                idx = (s1 - 512 if r & 1 else s0) + 512 * r
                assert np.array_equal(idx, slot(base + 512 * r))
                a[u][s][r] = lds[idx]
                accesses.append(idx)
    for u in range(groups):
        h = g0 + u
        for s in range(members):
            for r in range(1, 8):
                a[u][s][r] = a[u][s][r] * twiddle(64, h, r, inv)
        a[u] = transpose(dfts(a[u]), members, lanes)
        for s in range(members):
            for r in range(1, 8):
                a[u][s][r] = a[u][s][r] * twiddle(512, h + 64 * (m0 + ms * s), r, inv)
        a[u] = dfts(a[u])
    y = np.full(N, np.nan + 0j)
    for u in range(groups):
        for s in range(members):
            for r in range(8):
                y[g0 + u + 64 * (m0 + ms * s) + 512 * r] = a[u][s][r]
    return y, accesses


@pytest.mark.parametrize("groups,members", [(1, 1), (2, 1), (1, 2)],
                         ids=["wx1", "wx2", "wm2"])
@pytest.mark.parametrize("inv", [False, True], ids=["fwd", "bwd"])
def test_in_wave_exchange_layout_is_the_dft(groups, members, inv):
    rng = np.random.default_rng(4096 + groups + 2 * members)
    x = rng.standard_normal(N) + 1j * rng.standard_normal(N)
    y, accesses = emulate(x, groups, members, inv)
    want = np.fft.ifft(x) * N if inv else np.fft.fft(x)
    assert not np.isnan(y).any()
    assert np.linalg.norm(y - want) / np.linalg.norm(want) < 1e-13
    for acc in accesses:
        for w0 in range(0, len(acc), 32):
            assert len(set((acc[w0:w0 + 32] % 32).tolist())) == 32


def test_swizzles_are_bijections_that_keep_bits_5_and_up():
    i = np.arange(N)
    for slot in (slot_one_member, slot_two_members):
        s = slot(i)
        assert np.array_equal(np.sort(s), i)
        assert np.array_equal(s >> 5, i >> 5)
