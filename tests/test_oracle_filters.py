"""Pins of the oracle's 1D/2D building blocks against what the paper prints
and what the mathematics fixes (no GPU)."""
import numpy as np
import pytest

from oracle import filters as F
from tests.conftest import read_golden


def test_h_matches_printed_taps():
    # Section 5.1 footnote: five printed taps, 5 decimals
    printed = np.array([float(r[0]) for r in read_golden("h_shearlab_printed.txt")])
    h, o = F.qmf_maxflat9()
    assert o == 4 and len(h) == 9
    assert np.max(np.abs(h[:5] - printed)) < 5e-6
    assert np.allclose(h, h[::-1], atol=0, rtol=0)


def test_h_exact_closed_form():
    # the unique solution written with sqrt(2): H(w) = 1 + (8r-15)s^3 + (14-8r)s^4
    r = np.sqrt(2.0)
    exact = np.array([7 / 128 - r / 32, -13 / 64 + r / 8, (1 - r) / 8, 29 / 64 - r / 8,
                      9 / 64 + 5 * r / 16])
    h, _ = F.qmf_maxflat9()
    assert np.max(np.abs(h[:5] - exact)) < 1e-15
    w = np.linspace(0, np.pi, 101)
    s = np.sin(w / 2) ** 2
    H = F.dtft1d((h, 4), w / (2 * np.pi)).real
    assert np.max(np.abs(H - (1 + (8 * r - 15) * s ** 3 + (14 - 8 * r) * s ** 4))) < 1e-14


def test_h_orthonormality_bound():
    # Section 5.1: max_l |2 sum h(n)h(n+2l) - delta| <= 0.0018 (2 significant digits)
    bound = float(read_golden("orthonormality_bound.txt")[0][0])
    h, _ = F.qmf_maxflat9()
    vals = []
    for l in range(-4, 5):
        s = sum(h[n] * h[n + 2 * l] for n in range(9) if 0 <= n + 2 * l < 9)
        vals.append(abs(2 * s - (1.0 if l == 0 else 0.0)))
    assert abs(max(vals) - bound) < 5e-5


def test_h_properties():
    h = F.qmf_maxflat9()
    assert abs(h[0].sum() - 1.0) < 1e-15
    H = lambda xi: F.dtft1d(h, xi).real
    assert abs(H(0.5)) < 1e-15                          # zero at Nyquist
    assert abs(H(0.25) - 1 / np.sqrt(2)) < 1e-15        # 3 dB at half band
    xi = np.linspace(0, 0.5, 257)
    pc = H(xi) ** 2 + H(xi + 0.5) ** 2                   # power complementarity
    assert pc.min() > 0.9949 and pc.max() < 1.000011
    # two vanishing moments of the mirror filter (g sums to 0, first moment 0)
    g, o = F.mirror_highpass(h)
    n = np.arange(9) - o
    assert abs(g.sum()) < 1e-15 and abs((g * n).sum()) < 1e-15


def test_mirror_filter_is_half_shift():
    h = F.qmf_maxflat9()
    g = F.mirror_highpass(h)
    xi = np.linspace(-0.5, 0.5, 63)
    assert np.max(np.abs(F.dtft1d(g, xi) - F.dtft1d(h, xi + 0.5))) < 1e-14
    assert g[0][4] == h[0][4] > 0


@pytest.mark.parametrize("m", [1, 2, 3, 4, 5])
def test_cascade_lengths_and_products(m):
    h = F.qmf_maxflat9()
    g = F.mirror_highpass(h)
    hm = F.lowpass_cascade(h, m)
    gm = F.highpass_cascade(h, g, m)
    assert len(hm[0]) == 8 * (2 ** m - 1) + 1
    assert len(gm[0]) == 8 * (2 ** (m - 1)) + 8 * (2 ** (m - 1) - 1) + 1
    xi = np.linspace(-0.5, 0.5, 101)
    prod = np.ones_like(xi, dtype=complex)
    for k in range(m):
        prod *= F.dtft1d(h, 2 ** k * xi)
    assert np.max(np.abs(F.dtft1d(hm, xi) - prod)) < 1e-13         # eq. lowhigh
    hm1 = F.lowpass_cascade(h, m - 1)
    ref = F.dtft1d(g, 2 ** (m - 1) * xi) * F.dtft1d(hm1, xi)
    assert np.max(np.abs(F.dtft1d(gm, xi) - ref)) < 1e-13


@pytest.mark.parametrize("J", [1, 2, 3, 4, 5])
def test_littlewood_paley_1d(J):
    h = F.qmf_maxflat9()
    g = F.mirror_highpass(h)
    xi = np.linspace(0, 0.5, 2049)
    tot = np.abs(F.dtft1d(F.lowpass_cascade(h, J), xi)) ** 2
    for m in range(1, J + 1):
        tot += np.abs(F.dtft1d(F.highpass_cascade(h, g, m), xi)) ** 2
    assert tot.min() > 0.989 and tot.max() < 1.00002


def test_halfband_poly():
    P = np.polynomial.polynomial
    for K in (1, 2, 3, 4):
        c = F.halfband_poly(K)
        x = np.linspace(-1, 1, 41)
        v = P.polyval(x, c)
        assert np.max(np.abs(v + P.polyval(-x, c) - 1)) < 1e-14
        assert abs(P.polyval(1.0, c) - 1) < 1e-15 and abs(P.polyval(-1.0, c)) < 1e-15
    assert np.allclose(F.halfband_poly(2), [0.5, 0.75, 0.0, -0.25])


def test_fan_filter_properties():
    P = F.fan_filter(2)
    A, (o2, o1) = P
    assert A.shape == (7, 7) and (o2, o1) == (3, 3)
    assert np.allclose(A, A[::-1, ::-1], atol=0) and np.allclose(A, A[::-1, :], atol=0)
    # diamond support |n1| + |n2| <= 3
    n2, n1 = np.meshgrid(np.arange(7) - 3, np.arange(7) - 3, indexing="ij")
    assert np.all(A[np.abs(n1) + np.abs(n2) > 3] == 0)
    # half-band: P(eta) + P(eta swapped) = 1, i.e. taps + transposed taps = delta
    s = A + A.T
    d = np.zeros((7, 7)); d[3, 3] = 1
    assert np.max(np.abs(s - d)) < 1e-15
    e1, e2 = np.meshgrid(np.linspace(-0.5, 0.5, 81), np.linspace(-0.5, 0.5, 81))
    val = F.dtft2d(P, e1, e2)
    assert np.max(np.abs(val.imag)) < 1e-14
    x = (np.cos(2 * np.pi * e2) - np.cos(2 * np.pi * e1)) / 2
    assert np.max(np.abs(val.real - (1 + x) ** 2 * (2 - x) / 4)) < 1e-14
    # (cond2): |P|^2 bounded below on 1/4 < |eta1| < 1/2, |eta2/eta1| < 1
    region = (np.abs(e1) > 0.25) & (np.abs(e1) < 0.5) & (np.abs(e2) < np.abs(e1))
    assert np.min(np.abs(val[region]) ** 2) > 0.2
    assert abs(F.dtft2d(P, 0.5, 0.0).real - 1) < 1e-15 and abs(F.dtft2d(P, 0.0, 0.5).real) < 1e-15


def _lambda_d(h, d, xi1):
    L = 2 ** d
    hd = F.lowpass_cascade(h, d)
    return sum(np.abs(F.dtft1d(hd, (xi1 + r) / L)) ** 2 for r in range(L))


@pytest.mark.parametrize("d", [1, 2, 3, 4])
def test_shear_power_complementarity(d):
    h = F.qmf_maxflat9()
    lam = _lambda_d(h, d, np.linspace(-0.5, 0.5, 1001))
    assert lam.min() > 0.9938 and lam.max() < 1.000013


@pytest.mark.parametrize("d,m", [(1, 1), (1, -1), (2, 1), (1, 0), (2, 0)])
def test_integer_shear_special_case(d, m):
    # For k = m 2^d the digital shear is the integer shear (n1, n2) -> (n1 + m n2, n2)
    # filtered by Lambda_d(xi1) = sum_r |h_d((xi1 + r)/2^d)|^2 (eq. dshear2_alpha with
    # a shear that maps Z^2 to itself).
    h = F.qmf_maxflat9()
    rng = np.random.default_rng(d * 10 + m)
    A = rng.standard_normal((9, 7)); A = A + A[::-1, ::-1]
    f = (A, (4, 3))
    N = 64
    out = F.digital_shear(f, m * 2 ** d, d, h)
    hat = np.fft.fft2(F.periodize2d(out, N, N))
    base = np.fft.fft2(F.periodize2d(f, N, N))
    k1 = np.arange(N)
    lam = _lambda_d(h, d, k1 / N)
    # F_hat(xi1, xi2 - m xi1) on the grid: row index shifted by m * column index
    expect = np.empty_like(base)
    for c in range(N):
        expect[:, c] = np.roll(base[:, c], m * c) * lam[c]
    assert np.max(np.abs(hat - expect)) < 1e-12 * np.abs(base).max()


def test_shear_zero_is_near_identity():
    h = F.qmf_maxflat9()
    P = F.fan_filter(2)
    N = 64
    base = np.fft.fft2(F.periodize2d(P, N, N)).real
    for d in (1, 2):
        out = np.fft.fft2(F.periodize2d(F.digital_shear(P, 0, d, h), N, N)).real
        assert np.max(np.abs(out - base)) < 0.0062 * np.abs(base).max()
