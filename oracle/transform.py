"""Forward / inverse digital shearlet transform, thresholding, metrics (FP64).

TEST INFRASTRUCTURE ONLY (see the package docstring).

The undecimated transform is a circular convolution with each periodised
filter (Section 3.4, eq. convolution); by the convolution theorem it is a
pointwise product in the DFT domain (Section 4, Algorithm 1).  The inverse is
the dual-frame reconstruction (eqs. frame_filter, dual_filter, reconstruction;
Algorithm 2).  The filters are real and even, so no conjugation is needed.
"""
import numpy as np


def forward(x, filters):
    """c_i = IDFT(psi_hat_i * DFT(x)) for every filter (Algorithm 1)."""
    X = np.fft.fftn(np.asarray(x, dtype=np.float64))
    return np.stack([np.fft.ifftn(X * f).real for f in filters])


def forward_one(x, psi_hat):
    return np.fft.ifftn(np.fft.fftn(np.asarray(x, dtype=np.float64)) * psi_hat).real


def inverse(coeffs, filters, dual_weight):
    """x = IDFT( sum_i DFT(c_i) psi_hat_i / Psi_hat ) (Algorithm 2 with the
    dual filters of eq. dual_filter)."""
    acc = np.zeros(filters.shape[1:], dtype=np.complex128)
    for c, f in zip(coeffs, filters):
        acc += np.fft.fftn(np.asarray(c, dtype=np.float64)) * f
    return np.fft.ifftn(acc / dual_weight).real


def hard_threshold(c, delta):
    """(T_delta c)(n) = c(n) if |c(n)| >= delta else 0 (eq. hard_tresholding)."""
    c = np.asarray(c, dtype=np.float64)
    return np.where(np.abs(c) >= delta, c, 0.0)


def thresholds(system, sigma, K):
    """delta_i = K_j * sigma * ||psi_i||_2 per subband; the lowpass (index 0)
    is never thresholded (delta = 0).  K has one entry per scale."""
    norms = system.l2norms()
    out = np.zeros(system.R)
    for i, sb in enumerate(system.subbands):
        if sb.cone != 0:
            out[i] = K[sb.j] * sigma * norms[i]
    return out


def denoise(x, system, sigma, K):
    """T^-1 T_delta T x (Section 5.3) with per-scale constants K."""
    c = forward(x, system.filters)
    d = thresholds(system, sigma, K)
    ct = np.stack([hard_threshold(ci, di) for ci, di in zip(c, d)])
    return inverse(ct, system.filters, system.dual_weight)


def psnr(ref, est, peak=1.0):
    """PSNR = 20 log10(peak sqrt(N) / ||ref - est||_F) (eq. PSNR; the paper's
    255 becomes the image peak, 1 for images in [0, 1])."""
    ref = np.asarray(ref, dtype=np.float64)
    est = np.asarray(est, dtype=np.float64)
    err = np.linalg.norm((ref - est).ravel())
    return 20.0 * np.log10(peak * np.sqrt(ref.size) / err)


def circular_correlate_bruteforce(x, psi_per):
    """(x * psi_bar)(n) = sum_m x(m) psi(m - n) on the periodic grid, by the
    defining double sum (eq. convolution with psi_bar(n) = psi(-n))."""
    x = np.asarray(x, dtype=np.float64)
    out = np.zeros_like(x)
    for m in np.ndindex(*x.shape):
        if x[m] == 0.0:
            continue
        # psi(m - n) as an array over n: flip psi and roll so index n holds psi(m - n)
        flipped = np.flip(psi_per, axis=tuple(range(x.ndim)))
        flipped = np.roll(flipped, shift=tuple(mi + 1 for mi in m), axis=tuple(range(x.ndim)))
        out += x[m] * flipped
    return out


def circular_convolve_bruteforce(a, b):
    """(a (*) b)(n) = sum_m a(m) b(n - m) on the periodic grid, by the sum."""
    a = np.asarray(a, dtype=np.float64)
    out = np.zeros_like(a)
    for m in np.ndindex(*a.shape):
        if a[m] == 0.0:
            continue
        out += a[m] * np.roll(b, shift=m, axis=tuple(range(a.ndim)))
    return out
