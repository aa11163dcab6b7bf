"""2D and 3D digital shearlet filter banks, built as the paper constructs them.

TEST INFRASTRUCTURE ONLY (see the package docstring).

2D (Section 3.2.2, Definition digitSH_alpha; Section 3.4; Section 4.4):
  with d = d_j, L = 2^d and j = 0..J-1 (coarse to fine),
    p_j   = taps of P(2^{J-j-1} xi1, 2^{J-j+d} xi2)          (eq. ext_noshear_alpha)
    W_j   = g_{J-j} (x) h_{J-j+d}   (g along x1, h along x2)
    psi_{j,k} = S^d_{k/2^d}(p_j * W_j),   k = -L..L          (eq. 2dshear_filters)
  cone 2 swaps the variables; the lowpass is h_J (x) h_J (eq. frame_filter);
  cone 2 omits k = +-L unless full_system (Section 4.4).
3D (Section 3.3.2, Definition 3DdigitSH_alpha):
    Phi_{j,k} = S^d_{k/2^d}(h_{J-j+d} *_{x2} p_j)            (eq. 3Dfilters1_alpha)
    psi_hat_{j,k1,k2}(xi) = g_hat_{J-j}(xi1) Phi_hat_{j,k1}(xi1, xi2) Phi_hat_{j,k2}(xi1, xi3)
  pyramid 2 is psi_hat(xi2, xi1, xi3), pyramid 3 is psi_hat(xi3, xi1, xi2);
  pyramid 2 omits |k1| = L, pyramid 3 omits |k1| = L or |k2| = L.
Every spatial filter is periodised onto the grid and transformed with an FFT,
which samples its DTFT at the grid frequencies m/N.

Arrays: 2D grids are [N2, N1] (x1 fastest); 3D grids are [N3, N2, N1].
Subband order: lowpass first; then per scale j (coarse to fine) cone 1
(k = -L..L), cone 2; in 3D pyramids 1, 2, 3 with k1 outer, k2 inner.
"""
from dataclasses import dataclass, field

import numpy as np

from . import filters as F


@dataclass
class Subband:
    cone: int          # 0 = lowpass, 1/2 (2D cones) or 1/2/3 (3D pyramids)
    j: int             # scale, 0 = coarsest; -1 for the lowpass
    k1: int
    k2: int = 0


@dataclass
class ShearletSystem:
    dims: tuple                    # (N2, N1) or (N3, N2, N1)
    n_scales: int
    shear_levels: tuple
    full_system: bool
    subbands: list
    filters: np.ndarray            # [R, *dims] real FP64 psi_hat_i
    dual_weight: np.ndarray = field(default=None)   # Psi_hat = sum psi_hat_i^2

    @property
    def R(self):
        return len(self.subbands)

    def l2norms(self):
        """||psi_i^per||_2 = sqrt(mean_xi psi_hat_i^2) (Parseval)."""
        axes = tuple(range(1, self.filters.ndim))
        return np.sqrt(np.mean(self.filters ** 2, axis=axes))


def _dft2_real(spatial_per):
    hat = np.fft.fft2(spatial_per)
    scale = max(np.abs(hat).max(), 1e-300)
    if np.abs(hat.imag).max() > 1e-12 * scale:
        raise AssertionError("filter DFT is not real: filter not point-symmetric")
    return hat.real


def _components(qmf, dir_filter):
    h = qmf if qmf is not None else F.qmf_maxflat9()
    g = F.mirror_highpass(h)
    P = dir_filter if dir_filter is not None else F.fan_filter(2)
    return h, g, P


def wedge_2d(J, j, d, h, g, P):
    """p_j * W_j for scale j with shear level d (eq. ext_noshear_alpha)."""
    pj = F.upsample2d(P, 2 ** (J - j - 1), 2 ** (J - j + d))
    Wj = F.outer2d(F.lowpass_cascade(h, J - j + d), F.highpass_cascade(h, g, J - j))
    return F.conv2d(pj, Wj)


def spatial_filters_2d(n_scales, shear_levels, full_system=False, qmf=None, dir_filter=None):
    """Yield (Subband, spatial 2D filter) in subband order (finite support)."""
    J = n_scales
    h, g, P = _components(qmf, dir_filter)
    hJ = F.lowpass_cascade(h, J)
    yield Subband(0, -1, 0), F.outer2d(hJ, hJ)
    for j in range(J):
        d = int(shear_levels[j])
        L = 2 ** d
        wedge = wedge_2d(J, j, d, h, g, P)
        sheared = {k: F.digital_shear(wedge, k, d, h) for k in range(-L, L + 1)}
        for k in range(-L, L + 1):
            yield Subband(1, j, k), sheared[k]
        kr = range(-L, L + 1) if full_system else range(-L + 1, L)
        for k in kr:
            yield Subband(2, j, k), F.transpose2d(sheared[k])


def build_2d(dims, n_scales, shear_levels, full_system=False, qmf=None, dir_filter=None):
    N2, N1 = dims
    subs, hats = [], []
    for sb, filt in spatial_filters_2d(n_scales, shear_levels, full_system, qmf, dir_filter):
        subs.append(sb)
        hats.append(_dft2_real(F.periodize2d(filt, N2, N1)))
    filt = np.stack(hats)
    return ShearletSystem(tuple(dims), n_scales, tuple(shear_levels), full_system, subs,
                          filt, np.sum(filt ** 2, axis=0))


def spatial_filters_2d_periodized(dims, n_scales, shear_levels, full_system=False):
    """[R, N2, N1] periodised spatial filters psi_i^per (for brute force)."""
    N2, N1 = dims
    return np.stack([F.periodize2d(f, N2, N1)
                     for _, f in spatial_filters_2d(n_scales, shear_levels, full_system)])


# ---------------------------------------------------------------------------
# 3D
# ---------------------------------------------------------------------------

def phi_planes(J, j, d, h, P):
    """Spatial Phi_{j,k}, k = -L..L, on the (main, secondary) plane as 2D
    filters [secondary, main] (eq. 3Dfilters1_alpha, read with the h cascade
    along the secondary axis as in the parabolic case)."""
    L = 2 ** d
    pj = F.upsample2d(P, 2 ** (J - j - 1), 2 ** (J - j + d))
    base = F.conv2d(pj, F.along_x2(F.lowpass_cascade(h, J - j + d)))
    return {k: F.digital_shear(base, k, d, h) for k in range(-L, L + 1)}


def _plane_hat(phi, n_sec, n_main):
    """Phi_hat sampled on an [n_sec, n_main] grid, indexed [xi_sec, xi_main]."""
    return _dft2_real(F.periodize2d(phi, n_sec, n_main))


def _keep_3d(pyr, k1, k2, L, full):
    if full:
        return True
    if pyr == 2:
        return abs(k1) != L
    if pyr == 3:
        return abs(k1) != L and abs(k2) != L
    return True


def iter_filters_3d(dims, n_scales, shear_levels, full_system=False, qmf=None, dir_filter=None):
    """Yield (Subband, psi_hat [N3, N2, N1]) in subband order."""
    N3, N2, N1 = dims
    J = n_scales
    h, g, P = _components(qmf, dir_filter)
    hJ = F.lowpass_cascade(h, J)
    l1 = np.fft.fft(F.periodize1d(hJ, N1)).real
    l2 = np.fft.fft(F.periodize1d(hJ, N2)).real
    l3 = np.fft.fft(F.periodize1d(hJ, N3)).real
    yield Subband(0, -1, 0, 0), l3[:, None, None] * l2[None, :, None] * l1[None, None, :]
    for j in range(J):
        d = int(shear_levels[j])
        L = 2 ** d
        gJ = F.highpass_cascade(h, g, J - j)
        phis = phi_planes(J, j, d, h, P)
        ks = range(-L, L + 1)
        # pyramid 1: main axis x1; k1 shears toward x2, k2 toward x3
        gh = np.fft.fft(F.periodize1d(gJ, N1)).real
        A = {k: _plane_hat(phis[k], N2, N1) for k in ks}     # [xi2, xi1]
        B = {k: _plane_hat(phis[k], N3, N1) for k in ks}     # [xi3, xi1]
        for k1 in ks:
            for k2 in ks:
                if _keep_3d(1, k1, k2, L, full_system):
                    yield (Subband(1, j, k1, k2),
                           gh[None, None, :] * A[k1][None, :, :] * B[k2][:, None, :])
        # pyramid 2: psi_hat(xi2, xi1, xi3) = g(xi2) Phi_k1(xi2, xi1) Phi_k2(xi2, xi3)
        gh = np.fft.fft(F.periodize1d(gJ, N2)).real
        A = {k: _plane_hat(phis[k], N1, N2) for k in ks}     # [xi1, xi2]
        B = {k: _plane_hat(phis[k], N3, N2) for k in ks}     # [xi3, xi2]
        for k1 in ks:
            for k2 in ks:
                if _keep_3d(2, k1, k2, L, full_system):
                    yield (Subband(2, j, k1, k2),
                           gh[None, :, None] * A[k1].T[None, :, :] * B[k2][:, :, None])
        # pyramid 3: psi_hat(xi3, xi1, xi2) = g(xi3) Phi_k1(xi3, xi1) Phi_k2(xi3, xi2)
        gh = np.fft.fft(F.periodize1d(gJ, N3)).real
        A = {k: _plane_hat(phis[k], N1, N3) for k in ks}     # [xi1, xi3]
        B = {k: _plane_hat(phis[k], N2, N3) for k in ks}     # [xi2, xi3]
        for k1 in ks:
            for k2 in ks:
                if _keep_3d(3, k1, k2, L, full_system):
                    yield (Subband(3, j, k1, k2),
                           gh[:, None, None] * A[k1].T[:, None, :] * B[k2].T[:, :, None])


def build_3d(dims, n_scales, shear_levels, full_system=False, qmf=None, dir_filter=None):
    subs, hats = [], []
    for sb, hat in iter_filters_3d(dims, n_scales, shear_levels, full_system, qmf, dir_filter):
        subs.append(sb)
        hats.append(hat)
    filt = np.stack(hats)
    return ShearletSystem(tuple(dims), n_scales, tuple(shear_levels), full_system, subs,
                          filt, np.sum(filt ** 2, axis=0))


def dual_weight_3d(dims, n_scales, shear_levels, full_system=False):
    """Psi_hat accumulated without storing the filters (large systems)."""
    acc = np.zeros(dims)
    R = 0
    for _, hat in iter_filters_3d(dims, n_scales, shear_levels, full_system):
        acc += hat ** 2
        R += 1
    return acc, R


def build(dims, n_scales, shear_levels, full_system=False, qmf=None, dir_filter=None):
    if len(dims) == 2:
        return build_2d(dims, n_scales, shear_levels, full_system, qmf, dir_filter)
    if len(dims) == 3:
        return build_3d(dims, n_scales, shear_levels, full_system, qmf, dir_filter)
    raise ValueError("dims must have length 2 or 3")


def redundancy(ndim, shear_levels, full_system=False):
    """Number of filters R (Section 4.1, 4.4)."""
    R = 1
    for d in shear_levels:
        a = 2 * 2 ** d + 1
        if ndim == 2:
            R += 2 * a if full_system else 2 * a - 2
        else:
            R += 3 * a * a if full_system else 3 * a * a - 6 * a + 4
    return R
