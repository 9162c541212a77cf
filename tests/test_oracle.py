"""Pins of the FP64 oracle against what the DFT definition fixes.

Every check here comes from outside the oracle: closed forms of the DFT
(the paper, Section II-A), invariants (linearity, Parseval, inversion,
shift, symmetry), brute force between its two independent routes, and an
independent library (numpy's pocketfft).  The gradient is pinned by exact
central differences (the loss is quadratic) and by special cases.
"""
import numpy as np
import pytest

import oracle
from paper_2603_27569_amd import workloads

TOL = 1e-12


def _rand(n, batch=3, seed=7):
    g = np.random.default_rng(seed)
    return g.standard_normal((batch, n)) + 1j * g.standard_normal((batch, n))


def _close(a, b, tol):
    a = np.asarray(a)
    b = np.asarray(b)
    scale = max(1.0, float(np.max(np.abs(b))) if b.size else 1.0)
    assert np.max(np.abs(a - b)) <= tol * scale, np.max(np.abs(a - b))


ALL_DIRECT = [1, 2, 3, 4, 5, 7, 8, 12, 16, 64, 100]
ALL_FFT = [1, 2, 4, 8, 64, 128, 256, 1024, 4096, 2 ** 17]


def _roots(n, sign):
    m = np.arange(n)
    return np.exp(sign * 2j * np.pi * m / n)


@pytest.mark.parametrize("route,n", [("dft", n) for n in ALL_DIRECT] + [("fft", n) for n in ALL_FFT])
def test_delta_gives_constant(route, n):
    f = getattr(oracle, route)
    x = np.zeros(n, complex)
    x[0] = 1.0
    _close(f(x), np.ones(n), TOL)
    _close(f(x, inverse=True), np.ones(n), TOL)


@pytest.mark.parametrize("route,n", [("dft", n) for n in ALL_DIRECT] + [("fft", n) for n in ALL_FFT])
def test_shifted_delta(route, n):
    f = getattr(oracle, route)
    n0 = (3 * n) // 5
    x = np.zeros(n, complex)
    x[n0] = 1.0
    k = np.arange(n)
    expect = np.exp(-2j * np.pi * ((n0 * k) % n) / n)
    _close(f(x), expect, TOL)
    _close(f(x, inverse=True), np.conj(expect), TOL)


@pytest.mark.parametrize("route,n", [("dft", n) for n in ALL_DIRECT] + [("fft", n) for n in ALL_FFT])
def test_tone_single_bin(route, n):
    f = getattr(oracle, route)
    k0 = (37 + 5) % n
    m = np.arange(n)
    x = np.exp(2j * np.pi * ((k0 * m) % n) / n)
    expect = np.zeros(n, complex)
    expect[k0] = n
    _close(f(x), expect, TOL)


@pytest.mark.parametrize("route,n", [("dft", n) for n in ALL_DIRECT] + [("fft", n) for n in ALL_FFT])
def test_constant_and_ramp(route, n):
    f = getattr(oracle, route)
    c = 0.25 - 1.5j
    expect = np.zeros(n, complex)
    expect[0] = n * c
    _close(f(np.full(n, c)), expect, TOL)
    # Ramp x[m] = m: X[0] = n(n-1)/2, X[k] = n / (W^k - 1) for k != 0.
    x = np.arange(n, dtype=complex)
    w = np.exp(-2j * np.pi * np.arange(n) / n)
    expect = np.empty(n, complex)
    expect[0] = n * (n - 1) / 2.0
    expect[1:] = n / (w[1:] - 1.0)
    _close(f(x), expect, 1e-11)


def test_two_and_four_points():
    a, b, c, d = 1 + 2j, -0.5 + 0.25j, 3 - 1j, 0.125 + 4j
    _close(oracle.dft(np.array([a, b])), np.array([a + b, a - b]), TOL)
    expect = np.array([a + b + c + d, a - 1j * b - c + 1j * d,
                       a - b + c - d, a + 1j * b - c - 1j * d])
    _close(oracle.dft(np.array([a, b, c, d])), expect, TOL)
    _close(oracle.fft(np.array([a, b, c, d])), expect, TOL)
    # Backward direction flips the sign of i.
    expect_b = np.array([a + b + c + d, a + 1j * b - c - 1j * d,
                         a - b + c - d, a - 1j * b - c + 1j * d])
    _close(oracle.dft(np.array([a, b, c, d]), inverse=True), expect_b, TOL)


@pytest.mark.parametrize("n", [1, 2, 4, 8, 16, 32, 64, 128, 256, 512, 1024])
def test_recursive_equals_direct(n):
    x = _rand(n, 3, seed=n)
    for inv in (False, True):
        a = oracle.fft(x, inverse=inv)
        b = oracle.dft(x, inverse=inv)
        rel = np.linalg.norm(a - b) / np.linalg.norm(b)
        assert rel <= 1e-12, (n, inv, rel)


@pytest.mark.parametrize("n", [256, 512, 1024, 2048, 4096, 8192, 16384, 2 ** 15, 2 ** 18, 2 ** 20])
def test_numpy_cross_check(n):
    x = _rand(n, 2, seed=100 + n)
    f = oracle.fft(x)
    ref = np.fft.fft(x, axis=-1)
    assert np.linalg.norm(f - ref) / np.linalg.norm(ref) <= 1e-13
    b = oracle.fft(x, inverse=True)
    ref_b = np.fft.ifft(x, axis=-1) * n
    assert np.linalg.norm(b - ref_b) / np.linalg.norm(ref_b) <= 1e-13


@pytest.mark.parametrize("n", [16, 256, 4096, 2 ** 20])
def test_invariants(n):
    x = _rand(n, 1, seed=1)[0]
    y = _rand(n, 1, seed=2)[0]
    a, b = 0.3 - 1.1j, -2.0 + 0.5j
    F = oracle.fft
    # linearity
    _close(F(a * x + b * y), a * F(x) + b * F(y), 1e-12)
    # Parseval: sum |X|^2 = N sum |x|^2
    X = F(x)
    assert abs(np.sum(np.abs(X) ** 2) - n * np.sum(np.abs(x) ** 2)) <= 1e-12 * n * np.sum(np.abs(x) ** 2)
    # inversion: backward(forward(x)) = N x
    _close(F(X, inverse=True), n * x, 1e-12)
    # shift theorem: x[m - s] -> X[k] W^{s k}
    s = n // 3 + 1
    k = np.arange(n)
    _close(F(np.roll(x, s)), X * np.exp(-2j * np.pi * ((s * k) % n) / n), 1e-12)
    # conjugate symmetry of a real input: X[N-k] = conj X[k]
    r = F(x.real.astype(complex))
    _close(r[(-k) % n], np.conj(r), 1e-12)
    # F(conj x)[k] = conj X[-k mod N]
    _close(F(np.conj(x)), np.conj(X[(-k) % n]), 1e-12)


def test_batch_rows_independent():
    x = _rand(64, 5, seed=3)
    y = oracle.fft(x)
    for b in range(5):
        _close(y[b], oracle.fft(x[b]), 0.0 + 1e-15)


def test_complex64_inputs_promoted_exactly():
    x = workloads.plain_uniform(256, 4)
    y64 = oracle.fft(x)
    y128 = oracle.fft(x.astype(np.complex128))
    assert np.array_equal(y64, y128)


def test_rejects_bad_sizes():
    with pytest.raises(ValueError):
        oracle.fft(np.zeros(96, complex))  # > 64 and not a power of two
    assert oracle.dft(np.zeros(96, complex)).shape == (96,)


# ---------------------------------------------------------------- gradient

def _loss(x, w):
    return float(np.sum(oracle.spectral_energy(x, w)[0]))


@pytest.mark.parametrize("n", [64, 256])
def test_gradient_central_differences(n):
    """L is quadratic in x, so (L(x+hv)-L(x-hv))/2h is exact for any h."""
    g = np.random.default_rng(n)
    x = _rand(n, 2, seed=11)
    w = g.uniform(0, 1, n)
    _, grad = oracle.spectral_energy(x, w)
    idx = g.choice(x.size, size=12, replace=False)
    for i in idx:
        for comp in (1.0, 1j):
            e = np.zeros(x.size, complex)
            e[i] = comp
            e = e.reshape(x.shape)
            fd = (_loss(x + e, w) - _loss(x - e, w)) / 2.0
            got = grad.reshape(-1)[i].real if comp == 1.0 else grad.reshape(-1)[i].imag
            assert abs(fd - got) <= 1e-9 * max(1.0, np.max(np.abs(grad))), (i, comp, fd, got)


def test_gradient_unit_weight_closed_form():
    n = 512
    x = _rand(n, 3, seed=5)
    w = np.ones(n)
    loss, grad = oracle.spectral_energy(x, w)
    _close(grad, 2 * n * x, 1e-12)
    _close(loss, n * np.sum(np.abs(x) ** 2, axis=1), 1e-12)


def test_gradient_of_delta():
    n = 128
    g = np.random.default_rng(9)
    w = g.uniform(0, 1, n)
    x = np.zeros(n, complex)
    x[0] = 1.0
    loss, grad = oracle.spectral_energy(x, w)
    m = np.arange(n)
    # F^H(2 w^2)[m] = sum_k 2 w_k^2 exp(+2 pi i m k / N), written out as a sum
    expect = np.array([np.sum(2 * w ** 2 * np.exp(2j * np.pi * ((mm * m) % n) / n)) for mm in m])
    _close(grad.reshape(-1), expect, 1e-12)
    assert abs(loss[0] - np.sum(w ** 2)) <= 1e-12 * n


def test_loss_matches_library_spectrum():
    n = 1024
    x = _rand(n, 2, seed=21)
    w = np.random.default_rng(3).uniform(0, 1, n)
    loss, _ = oracle.spectral_energy(x, w)
    ref = np.sum((w ** 2) * np.abs(np.fft.fft(x, axis=-1)) ** 2, axis=1)
    _close(loss, ref, 1e-12)


# ----------------------------------------------------------- matched filter

def test_matched_filter_identity_and_shift():
    n = 256
    x = _rand(n, 2, seed=31)
    _close(oracle.matched_filter(x, np.ones(n)), x, 1e-12)
    # H = F(delta[m - s]) -> conj(H) X = F(x[m + s]) -> out[m] = x[m + s]
    s = 37
    k = np.arange(n)
    h = np.exp(-2j * np.pi * ((s * k) % n) / n)
    _close(oracle.matched_filter(x, h), np.roll(x, -s, axis=-1), 1e-12)


def test_matched_filter_is_circular_cross_correlation():
    n = 64
    g = np.random.default_rng(41)
    x = _rand(n, 1, seed=42)[0]
    hs = g.standard_normal(n) + 1j * g.standard_normal(n)
    h = np.fft.fft(hs)
    out = oracle.matched_filter(x, h)
    expect = np.array([np.sum(np.conj(hs) * np.roll(x, -m)) for m in range(n)])
    _close(out, expect, 1e-12)
