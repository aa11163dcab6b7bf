"""Inpainting by iterative hard thresholding (Section 5, "Image Inpainting",
Algorithm 3; "Video Inpainting" runs the same scheme on volumes).  FP64.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Given the occluded signal f_masked = M .* f and the binary mask M (1 where the
signal is known), Algorithm 3 starts from f_inp = 0 and a threshold
delta = delta_init, and repeats `iterations` times:

    f_res = M .* (f_masked - f_inp)
    f_inp = T^-1 T_delta T (f_res + f_inp)
    delta = lambda * delta,    lambda = delta_min ** (1 / (iterations - 1))

so the last iteration thresholds at delta_init * delta_min.

Readings of points the paper leaves open:
  * T_delta is the hard-thresholding operator of eq. hard_tresholding applied
    as in the denoising experiment: subband i is thresholded at
    delta * ||psi_i||_2 (the coefficient's own scale) and the lowpass is
    kept.  The schedule therefore runs over normalised thresholds.
  * delta_min is a ratio (the printed lambda does not involve delta_init),
    so the last threshold is delta_init * delta_min; one iteration uses
    delta_init alone.
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


def step(f_inp, f_masked, mask, system, delta):
    """One pass of the loop body of Algorithm 3."""
    m = np.asarray(mask, dtype=np.float64)
    f_res = m * (np.asarray(f_masked, dtype=np.float64) - f_inp)
    c = T.forward(f_res + f_inp, system.filters)
    return T.inverse(threshold_all(c, system, delta), system.filters, system.dual_weight)


def inpaint(f_masked, mask, system, delta_init, delta_min, iterations, f_start=None, t_begin=0,
            t_end=None):
    """Algorithm 3.  With t_begin / t_end only iterations t_begin..t_end-1 of
    the `iterations`-step schedule run, starting from f_start (the state
    after t_begin iterations; zero when t_begin = 0)."""
    deltas = schedule(delta_init, delta_min, iterations)
    t_end = iterations if t_end is None else t_end
    f = np.zeros(np.shape(f_masked)) if t_begin == 0 or f_start is None else \
        np.asarray(f_start, dtype=np.float64).copy()
    for t in range(t_begin, t_end):
        f = step(f, f_masked, mask, system, deltas[t])
    return f
