"""Image decomposition by iterative thresholding with two transforms
(Section 5, "Image Decomposition", Algorithm 4) and the undecimated
separable wavelet transform it pairs with the shearlets.  FP64.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Wavelet bank (Section 3.4, the 2D digital wavelet transform built from the
cascades of eq. lowhigh, without the subsampling by 2^{J-j}): subband order
lowpass h_J (x) h_J, then for j = 0..J-1 (coarse to fine)
    cone 1: g_{J-j} along x1, h_{J-j} along x2,
    cone 2: h_{J-j} along x1, g_{J-j} along x2,
    cone 3: g_{J-j} along both,
built spatially (upsampled convolution cascades, tensor products,
periodisation, DFT) like the shearlet filters.

Algorithm 4 splits f into two parts, each sparse in one of two transforms
(here the shearlets for curve-like content and the wavelets for point-like
content).  Both parts start at zero.  In every pass each part is re-estimated
by hard-threshold denoising, in its own transform, of what the other part
leaves of f, i.e. f minus the other part's estimate from the start of the
pass; both parts are updated from the same starting estimates.  The
threshold follows the geometric schedule of Algorithm 3.  Readings: either
system thresholds subband i at delta ||psi_i||_2 and keeps its lowpass (as
in inpainting); the optional total-variation correction the paper mentions
is not applied.
"""
import numpy as np

from . import filters as F
from . import inpaint as I
from . import system as S
from . import transform as T


def spatial_wavelet_filters_2d(n_scales, qmf=None):
    """Yield (Subband, spatial 2D filter [x2, x1]) of the wavelet bank."""
    J = n_scales
    h = qmf if qmf is not None else F.qmf_maxflat9()
    g = F.mirror_highpass(h)
    hJ = F.lowpass_cascade(h, J)
    yield S.Subband(0, -1, 0), F.outer2d(hJ, hJ)
    for j in range(J):
        hj = F.lowpass_cascade(h, J - j)
        gj = F.highpass_cascade(h, g, J - j)
        yield S.Subband(1, j, 0), F.outer2d(hj, gj)
        yield S.Subband(2, j, 0), F.outer2d(gj, hj)
        yield S.Subband(3, j, 0), F.outer2d(gj, gj)


def build_wavelet_2d(dims, n_scales, qmf=None):
    N2, N1 = dims
    subs, hats = [], []
    for sb, filt in spatial_wavelet_filters_2d(n_scales, qmf):
        subs.append(sb)
        hats.append(S._dft2_real(F.periodize2d(filt, N2, N1)))
    filt = np.stack(hats)
    return S.ShearletSystem(tuple(dims), n_scales, (0,) * n_scales, False, subs, filt,
                            np.sum(filt ** 2, axis=0))


def decompose(f, sys0, sys1, delta_init, delta_min, iterations, start=None, t_begin=0,
              t_end=None):
    """Algorithm 4: returns the two parts (f0, f1).  With t_begin / t_end only
    passes t_begin..t_end-1 of the schedule run, from start = (f0, f1) after
    t_begin passes (zeros when t_begin = 0)."""
    f = np.asarray(f, dtype=np.float64)
    deltas = I.schedule(delta_init, delta_min, iterations)
    t_end = iterations if t_end is None else t_end
    if t_begin == 0 or start is None:
        f0, f1 = np.zeros(f.shape), np.zeros(f.shape)
    else:
        f0, f1 = (np.asarray(a, dtype=np.float64).copy() for a in start)
    for t in range(t_begin, t_end):
        # both parts from the estimates at the start of the pass
        f0, f1 = (I.denoise_at(f - f1, sys0, deltas[t]),
                  I.denoise_at(f - f0, sys1, deltas[t]))
    return f0, f1
