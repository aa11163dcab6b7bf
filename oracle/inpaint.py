"""Inpainting by iterative hard thresholding (Section 5, image inpainting,
Algorithm 3; video inpainting applies the same scheme to volumes).  FP64.

TEST INFRASTRUCTURE ONLY (see the package docstring).

The method is a fixed-point iteration with a shrinking threshold.  The
estimate starts at zero.  Each pass first merges the observation with the
estimate: samples the mask marks as known take their observed value, the
others keep the current estimate.  The merged signal is then denoised by
hard thresholding in the shearlet domain (forward transform, threshold,
dual-frame inverse), and the result becomes the new estimate.  The threshold
starts at delta_init and is multiplied by the same ratio after every pass,
the ratio being chosen so that the last pass thresholds at
delta_init * delta_min.

Readings of points the paper leaves open:
  * the threshold operator is the one of eq. hard_tresholding used as in the
    denoising experiment: subband i is thresholded at delta * ||psi_i||_2
    (the coefficient's own scale) and the lowpass is kept, so the schedule
    runs over normalised thresholds;
  * delta_min is a ratio (the printed decay factor does not involve
    delta_init), so the last threshold is delta_init * delta_min; a single
    pass uses delta_init alone;
  * the mask is binary (1 = known); the merge M f_masked + (1 - M) f is then
    an exact selection.
"""
import numpy as np

from . import transform as T


def schedule(delta_init, delta_min, iterations):
    """Thresholds delta_t, t = 0..iterations-1 (geometric, ratio lambda)."""
    if iterations < 1:
        raise ValueError("iterations must be >= 1")
    lam = float(delta_min) ** (1.0 / (iterations - 1)) if iterations > 1 else 1.0
    out, d = [], float(delta_init)
    for _ in range(iterations):
        out.append(d)
        d = lam * d
    return out


def threshold_all(c, system, delta):
    """T_delta on every subband: |c_i| >= delta ||psi_i||_2 kept, lowpass kept."""
    d = T.thresholds(system, delta, np.ones(max(sb.j for sb in system.subbands) + 1))
    return np.stack([T.hard_threshold(ci, di) for ci, di in zip(c, d)])


def merge_known(f_est, f_masked, mask):
    """Observed values on the known samples, the estimate elsewhere:
    M f_masked + (1 - M) f_est (an exact selection for a binary mask)."""
    m = np.asarray(mask, dtype=np.float64)
    return m * np.asarray(f_masked, dtype=np.float64) + (1.0 - m) * f_est


def denoise_at(g, system, delta):
    """Hard-threshold denoising of g at the normalised threshold delta."""
    c = threshold_all(T.forward(g, system.filters), system, delta)
    return T.inverse(c, system.filters, system.dual_weight)


def step(f_est, f_masked, mask, system, delta):
    """One pass of Algorithm 3: merge, then denoise at delta."""
    return denoise_at(merge_known(f_est, f_masked, mask), system, delta)


def inpaint(f_masked, mask, system, delta_init, delta_min, iterations, f_start=None, t_begin=0,
            t_end=None):
    """Algorithm 3: `iterations` passes from a zero estimate.  With t_begin /
    t_end only passes t_begin..t_end-1 of the schedule run, starting from
    f_start (the estimate after t_begin passes; zero when t_begin = 0)."""
    deltas = schedule(delta_init, delta_min, iterations)
    t_end = iterations if t_end is None else t_end
    f = np.zeros(np.shape(f_masked)) if t_begin == 0 or f_start is None else \
        np.asarray(f_start, dtype=np.float64).copy()
    for t in range(t_begin, t_end):
        f = step(f, f_masked, mask, system, deltas[t])
    return f
