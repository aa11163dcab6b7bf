"""Pins of the oracle's inpainting (Algorithm 3) against what the mathematics
fixes, no GPU: the schedule's closed form, the limits delta = 0 (the loop is
the identity on the known samples) and delta = inf (only the lowpass
survives), the Gaussian statistics of normalised thresholds, a brute-force
evaluation of the iteration with convolution sums, and the paper's
qualitative claim (the synthesis approaches the original on the known
samples)."""
import math

import numpy as np
import pytest

from oracle import inpaint as I
from oracle import system as S
from oracle import transform as T
from paper_1402_5670_amd import synthetic as syn


def test_schedule_closed_form():
    # lambda = delta_min^(1/(iterations-1)): delta_0 = delta_init and after
    # iterations-1 multiplications delta = delta_init * delta_min
    d = I.schedule(4.0, 0.005, 300)
    assert len(d) == 300 and d[0] == 4.0
    assert abs(d[-1] - 4.0 * 0.005) < 1e-12
    r = np.array(d[1:]) / np.array(d[:-1])
    assert np.max(np.abs(r - 0.005 ** (1 / 299))) < 1e-14
    assert I.schedule(2.0, 0.1, 2) == [2.0, 0.2]
    assert I.schedule(3.0, 0.1, 1) == [3.0]
    with pytest.raises(ValueError):
        I.schedule(1.0, 0.1, 0)


def test_full_mask_without_threshold_is_identity():
    # M = 1 and delta = 0: f_res + f_inp = f_masked every iteration and T^-1 T
    # is exact, so every iterate equals the signal (a sign error in f_res or a
    # dropped "+ f_inp" fails from the first or second iteration on)
    sysm = S.build_2d((32, 48), 2, [1, 1])
    x = np.random.default_rng(31).standard_normal((32, 48))
    ones = np.ones(x.shape)
    for its in (1, 2, 3):
        assert np.max(np.abs(I.inpaint(x, ones, sysm, 0.0, 1.0, its) - x)) < 1e-12


def test_zero_threshold_keeps_known_samples():
    # delta = 0: the first iterate is T^-1 T (M f) = M f, and M f is a fixed
    # point since M (M f - M f) = 0 for a binary M; a mask that is not
    # symmetric catches a transposed or complemented M
    sysm = S.build_2d((32, 32), 2, [1, 1])
    clean, m = syn.inpainting_case(32, 32, 5, "random")
    m[0, :8] = 1
    m[:8, 0] = 0
    fm = clean * m
    for its in (1, 3):
        assert np.max(np.abs(I.inpaint(fm, m, sysm, 0.0, 1.0, its) - fm)) < 1e-12


def test_infinite_threshold_keeps_only_the_lowpass():
    # delta = inf removes every detail coefficient; the lowpass is kept, so one
    # iteration on a full mask is IDFT(DFT(x) phi_hat^2 / Psi_hat)
    sysm = S.build_2d((32, 32), 2, [1, 1])
    x = np.random.default_rng(32).standard_normal((32, 32))
    out = I.inpaint(x, np.ones(x.shape), sysm, np.inf, 1.0, 1)
    ref = np.fft.ifft2(np.fft.fft2(x) * sysm.filters[0] ** 2 / sysm.dual_weight).real
    assert np.max(np.abs(out - ref)) < 1e-12


def test_normalised_threshold_statistics():
    # For white Gaussian noise of unit variance every coefficient of subband i
    # is N(0, ||psi_i||_2^2).  Thresholding at delta ||psi_i||_2 therefore zeroes
    # the fraction erf(delta / sqrt 2) of every detail subband (0.6827 at
    # delta = 1); thresholds that ignored the subband norms would give 0.52 ..
    # 0.85 on this system.
    sysm = S.build_2d((256, 256), 2, [1, 1])
    x = np.random.default_rng(21).standard_normal((256, 256))
    ct = I.threshold_all(T.forward(x, sysm.filters), sysm, 1.0)
    target = math.erf(1 / math.sqrt(2))
    for i in range(1, sysm.R):
        assert abs(np.mean(ct[i] == 0.0) - target) < 0.03, i
    assert np.count_nonzero(ct[0]) == ct[0].size


def _bruteforce_step(f, fm, m, per, dual_per, l2, delta):
    # the loop body with every convolution evaluated as its defining sum:
    # analysis c_i = g * psi_bar_i, synthesis x = sum_i c_i (*) psi_tilde_i
    g = m * (fm - f) + f
    out = np.zeros_like(f)
    for i in range(len(per)):
        c = T.circular_correlate_bruteforce(g, per[i])
        if i > 0:
            c = np.where(np.abs(c) >= delta * l2[i], c, 0.0)
        out += T.circular_convolve_bruteforce(c, dual_per[i])
    return out


def test_bruteforce_iterations():
    # two iterations on a 16 x 16 grid by convolution sums against the FFT route
    dims = (16, 16)
    sysm = S.build_2d(dims, 2, [1, 1])
    per = S.spatial_filters_2d_periodized(dims, 2, [1, 1])
    dual_per = np.stack([np.fft.ifft2(f / sysm.dual_weight).real for f in sysm.filters])
    l2 = np.sqrt(np.sum(per ** 2, axis=(1, 2)))
    clean, m = syn.inpainting_case(16, 16, 9, "random")
    fm = clean * m
    d = I.schedule(1.0, 0.1, 2)
    f = np.zeros(dims)
    for t in range(2):
        f = _bruteforce_step(f, fm, m, per, dual_per, l2, d[t])
    got = I.inpaint(fm, m, sysm, 1.0, 0.1, 2)
    assert np.max(np.abs(got - f)) < 1e-12
    assert np.max(np.abs(f)) > 0.1          # not a trivial all-zero case


def test_segments_compose():
    # running iterations 0..k-1 and then k..n-1 from that state is the full run
    sysm = S.build_2d((32, 32), 2, [1, 1])
    clean, m = syn.inpainting_case(32, 32, 6, "squares")
    fm = clean * m
    full = I.inpaint(fm, m, sysm, 4.0, 0.01, 6)
    a = I.inpaint(fm, m, sysm, 4.0, 0.01, 6, t_end=2)
    b = I.inpaint(fm, m, sysm, 4.0, 0.01, 6, f_start=a, t_begin=2)
    assert np.max(np.abs(full - b)) < 1e-13


@pytest.mark.parametrize("kind", ["random", "squares", "text"])
def test_inpainting_recovers_cartoon(kind):
    # the iterates approach the original on the known samples while filling
    # the missing ones (Section 5, image inpainting): PSNR well above the
    # occluded input and small error where M = 1
    n = 64
    sysm = S.build_2d((n, n), 2, [1, 1])
    clean, m = syn.inpainting_case(n, n, 12, kind)
    fm = clean * m
    f = I.inpaint(fm, m, sysm, 4.0, 0.005, 40)
    assert T.psnr(clean, f) > T.psnr(clean, fm) + 6.0
    known = m == 1
    assert np.max(np.abs(f - clean)[known]) < 0.1
    assert np.sqrt(np.mean((f - clean)[known] ** 2)) < 0.02
