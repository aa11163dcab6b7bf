"""Quality measures used to report results (not part of the transform).

psnr    eq. PSNR with the peak of images in [0, 1]
q_value Q(f0_est, delta) of the image decomposition experiment (Section 5):
        ||G * f0 - G * B_delta(f0_est)||_2 / ||G * f0||_2, B_delta the
        binarisation |v| >= delta and G a sampled Gaussian (standard deviation
        2 pixels, 13 x 13 taps, unit sum; the paper does not print its
        filter), applied as a periodic convolution
q_opt   min of Q over delta in {0, 1/255, ..., 1} (the paper's {0..255} for
        8-bit images)
"""
import numpy as np

GAUSS_SIGMA = 2.0
GAUSS_RADIUS = 6


def psnr(ref, est):
    ref = np.asarray(ref, dtype=np.float64)
    err = np.linalg.norm((ref - np.asarray(est, dtype=np.float64)).ravel())
    return float(20.0 * np.log10(np.sqrt(ref.size) / err))


def gaussian_kernel(sigma=GAUSS_SIGMA, radius=GAUSS_RADIUS):
    t = np.arange(-radius, radius + 1, dtype=np.float64)
    g1 = np.exp(-0.5 * (t / sigma) ** 2)
    k = np.outer(g1, g1)
    return k / k.sum()


def _kernel_hat(shape, kernel):
    H, W = shape
    r = kernel.shape[0] // 2
    per = np.zeros((H, W))
    for dy in range(-r, r + 1):
        for dx in range(-r, r + 1):
            per[dy % H, dx % W] += kernel[dy + r, dx + r]
    return np.fft.rfft2(per)


def _q(ref_b, b, khat, shape):
    blurred = np.fft.irfft2(np.fft.rfft2(b) * khat, s=shape)
    return float(np.linalg.norm((ref_b - blurred).ravel()) / np.linalg.norm(ref_b.ravel()))


def q_value(f0_true, f0_est, delta, kernel=None):
    kernel = gaussian_kernel() if kernel is None else kernel
    f0_true = np.asarray(f0_true, dtype=np.float64)
    khat = _kernel_hat(f0_true.shape, kernel)
    ref_b = np.fft.irfft2(np.fft.rfft2(f0_true) * khat, s=f0_true.shape)
    b = (np.abs(np.asarray(f0_est, dtype=np.float64)) >= delta).astype(np.float64)
    return _q(ref_b, b, khat, f0_true.shape)


def q_opt(f0_true, f0_est):
    """(min_delta Q, the minimising delta)."""
    f0_true = np.asarray(f0_true, dtype=np.float64)
    a = np.abs(np.asarray(f0_est, dtype=np.float64))
    khat = _kernel_hat(f0_true.shape, gaussian_kernel())
    ref_b = np.fft.irfft2(np.fft.rfft2(f0_true) * khat, s=f0_true.shape)
    vals = [_q(ref_b, (a >= d / 255.0).astype(np.float64), khat, f0_true.shape)
            for d in range(256)]
    k = int(np.argmin(vals))
    return vals[k], k / 255.0
