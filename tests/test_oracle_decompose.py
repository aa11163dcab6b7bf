"""Pins of the oracle's wavelet bank and image decomposition (Algorithm 4),
and of the Q measure, against what the mathematics fixes (no GPU)."""
import numpy as np
import pytest

from oracle import decompose as D
from oracle import filters as F
from oracle import system as S
from oracle import transform as T
from paper_1402_5670_amd import metrics as M
from paper_1402_5670_amd import synthetic as syn


def test_wavelet_perfect_reconstruction_and_frame():
    for dims, J in (((32, 48), 2), ((64, 64), 3)):
        sysw = D.build_wavelet_2d(dims, J)
        assert sysw.R == 3 * J + 1
        x = np.random.default_rng(41).standard_normal(dims)
        c = T.forward(x, sysw.filters)
        assert np.max(np.abs(T.inverse(c, sysw.filters, sysw.dual_weight) - x)) < 1e-12
        # the squared filters telescope to 1 for a power-complementary pair;
        # h_ShearLab misses that by at most 0.0051 (|H|^2 + |G|^2 in
        # [0.99491, 1.00001]), so every level keeps the sum within [0.97, 1.0001]
        assert sysw.dual_weight.min() > 0.97 and sysw.dual_weight.max() < 1.0001


def test_wavelet_axes():
    # a signal constant along x2 has its spectrum on xi2 = 0, where every
    # g cascade vanishes (g_hat(0) = 0): cone 2 (g along x2) and cone 3 are zero,
    # cone 1 (g along x1) is not
    dims, J = (32, 64), 3
    sysw = D.build_wavelet_2d(dims, J)
    s = np.random.default_rng(42).standard_normal(dims[1])
    x = np.tile(s, (dims[0], 1))
    c = T.forward(x, sysw.filters)
    for i, sb in enumerate(sysw.subbands):
        if sb.cone in (2, 3):
            assert np.max(np.abs(c[i])) < 1e-12
        elif sb.cone == 1:
            assert np.max(np.abs(c[i])) > 1e-2


def _mallat_1d(s, h, g, m):
    """Decimated DWT detail at level m: (filter h, keep even samples) m-1
    times, then filter g and keep even samples; periodic, taps centred on
    their origin."""
    def filt_down(a, f):
        taps, o = f
        out = np.zeros(len(a))
        for t, tap in enumerate(taps):
            out += tap * np.roll(a, t - o)
        return out[::2]
    a = np.asarray(s, dtype=np.float64)
    for _ in range(m - 1):
        a = filt_down(a, h)
    return filt_down(a, g)


def test_undecimated_equals_mallat_cascade_on_the_subsampled_grid():
    # eq. owt: <f, psi_{j,m}> = (w_bar_j * f)(2^{J-j} m) with w_j = g_{J-j}: the
    # undecimated subband sampled every 2^{J-j} samples is the Mallat pyramid's
    # detail (noble identities), here along x1 for a signal constant along x2
    # (the x2 factor h_{J-j} then contributes its DC gain, 1)
    dims, J = (16, 64), 3
    sysw = D.build_wavelet_2d(dims, J)
    h = F.qmf_maxflat9()
    g = F.mirror_highpass(h)
    s = np.random.default_rng(43).standard_normal(dims[1])
    c = T.forward(np.tile(s, (dims[0], 1)), sysw.filters)
    checked = 0
    for i, sb in enumerate(sysw.subbands):
        if sb.cone != 1:
            continue
        m = J - sb.j
        ref = _mallat_1d(s, h, g, m)
        assert np.max(np.abs(c[i][0, ::2 ** m] - ref)) < 1e-12, sb
        assert np.max(np.abs(c[i][0, 1::2 ** m] - ref)) > 1e-3   # phase matters
        checked += 1
    assert checked == J


def _lowpass_multiplier(sysm):
    return sysm.filters[0] ** 2 / sysm.dual_weight


def test_decompose_limits():
    dims = (32, 32)
    s0 = S.build_2d(dims, 2, [1, 1])
    s1 = D.build_wavelet_2d(dims, 2)
    f = np.random.default_rng(44).standard_normal(dims)
    # delta = 0: no thresholding, T^-1 T = I: (f, f), then f_res = -f gives (0, 0)
    a0, a1 = D.decompose(f, s0, s1, 0.0, 1.0, 1)
    assert np.max(np.abs(a0 - f)) < 1e-12 and np.max(np.abs(a1 - f)) < 1e-12
    b0, b1 = D.decompose(f, s0, s1, 0.0, 1.0, 2)
    assert np.max(np.abs(b0)) < 1e-12 and np.max(np.abs(b1)) < 1e-12
    # delta = inf: each part keeps only its own lowpass, L0 = phi0^2/Psi0 and
    # L1 = phi1^2/Psi1 as Fourier multipliers.  Iteration 1: f0 = L0 f,
    # f1 = L1 f.  Iteration 2 (both from the same f_res):
    # f0 = L0 (1 - L1) f, f1 = L1 (1 - L0) f.
    X = np.fft.fft2(f)
    L0, L1 = _lowpass_multiplier(s0), _lowpass_multiplier(s1)
    c0, c1 = D.decompose(f, s0, s1, np.inf, 1.0, 1)
    assert np.max(np.abs(c0 - np.fft.ifft2(L0 * X).real)) < 1e-12
    assert np.max(np.abs(c1 - np.fft.ifft2(L1 * X).real)) < 1e-12
    d0, d1 = D.decompose(f, s0, s1, np.inf, 1.0, 2)
    assert np.max(np.abs(d0 - np.fft.ifft2(L0 * (1 - L1) * X).real)) < 1e-12
    assert np.max(np.abs(d1 - np.fft.ifft2(L1 * (1 - L0) * X).real)) < 1e-12


def test_decompose_segments_compose():
    dims = (32, 32)
    s0 = S.build_2d(dims, 2, [1, 1])
    s1 = D.build_wavelet_2d(dims, 2)
    c, p = syn.points_and_curves(32, 32, 5)
    f = c + p
    full = D.decompose(f, s0, s1, 2.0, 0.05, 5)
    a = D.decompose(f, s0, s1, 2.0, 0.05, 5, t_end=2)
    b = D.decompose(f, s0, s1, 2.0, 0.05, 5, start=a, t_begin=2)
    assert max(np.max(np.abs(full[k] - b[k])) for k in range(2)) < 1e-13


def test_decompose_separates_points_and_curves():
    # the shearlet part approaches the curves and the wavelet part the points
    # (Section 5, image decomposition): Q well below that of the unseparated image
    n = 128
    s0 = S.build_2d((n, n), 3, [1, 1, 2])
    s1 = D.build_wavelet_2d((n, n), 3)
    c, p = syn.points_and_curves(n, n, 3)
    f = c + p
    f0, f1 = D.decompose(f, s0, s1, 2.0, 0.05, 40)
    qc, qp = M.q_opt(c, f0)[0], M.q_opt(p, f1)[0]
    qc_triv, qp_triv = M.q_opt(c, f)[0], M.q_opt(p, f)[0]
    assert qc < 0.6 * qc_triv and qc < 0.25
    assert qp < 0.2 * qp_triv and qp < 0.5


def test_q_measure():
    k = M.gaussian_kernel()
    assert abs(k.sum() - 1.0) < 1e-14 and np.allclose(k, k.T) and np.allclose(k, k[::-1, ::-1])
    c, _ = syn.points_and_curves(64, 64, 8)
    # a binary estimate equal to the truth: Q = 0 for every delta in (0, 1]
    assert M.q_value(c, c, 0.5) < 1e-12 and M.q_opt(c, c)[0] < 1e-12
    # an empty estimate: Q = ||G f0|| / ||G f0|| = 1
    assert abs(M.q_value(c, np.zeros_like(c), 0.5) - 1.0) < 1e-12
    # B_delta depends on |v| >= delta only: sign and values above delta do not matter
    assert abs(M.q_value(c, -3.0 * c, 0.5)) < 1e-12
    # the blur is a periodic convolution: a circular shift of both arguments
    # leaves Q unchanged
    e = c + 0.3 * np.random.default_rng(9).random(c.shape)
    q1 = M.q_value(c, e, 0.4)
    q2 = M.q_value(np.roll(c, (5, -7), (0, 1)), np.roll(e, (5, -7), (0, 1)), 0.4)
    assert abs(q1 - q2) < 1e-12


@pytest.mark.parametrize("seed", [1, 2])
def test_points_and_curves_generator(seed):
    c, p = syn.points_and_curves(256, 256, seed)
    assert set(np.unique(c)) <= {0.0, 1.0} and set(np.unique(p)) <= {0.0, 1.0}
    assert 0.005 < c.mean() < 0.1 and 0.001 < p.mean() < 0.05
