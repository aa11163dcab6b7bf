"""Pins of the oracle's filter banks and transforms (no GPU): the paper's
counts and frame-bound table, perfect reconstruction, brute-force circular
convolution, symmetry and support invariants."""
import numpy as np
import pytest

from oracle import filters as F
from oracle import system as S
from oracle import transform as T
from tests.conftest import read_golden


def _table():
    out = {}
    for name, ndim, levels, dirs, R, A, BA in read_golden("frame_bounds_table.txt"):
        out[name] = dict(ndim=int(ndim), levels=[int(v) for v in levels.split(",")],
                         dirs=[int(v) for v in dirs.split(",")], R=int(R), A=float(A),
                         BA=float(BA))
    return out


def test_counts_match_paper_table():
    # Section 4.1 (R formula), Section 4.4 (omission) and the Section 5.1 table
    for name, row in _table().items():
        if row["ndim"] == 2:
            subs = [sb for sb, _ in S.spatial_filters_2d(len(row["levels"]), row["levels"])]
            per_scale = [sum(1 for s in subs if s.j == j) for j in range(len(row["levels"]))]
            assert per_scale == row["dirs"]
            assert len(subs) == row["R"]
            for j, d in enumerate(row["levels"]):
                assert per_scale[j] == 2 ** (d + 2)
        else:
            subs = [sb for sb, _ in S.iter_filters_3d((8, 8, 8), len(row["levels"]), row["levels"])]
            per_scale = [sum(1 for s in subs if s.j == j) for j in range(len(row["levels"]))]
            assert per_scale == row["dirs"]
            assert len(subs) == row["R"]


def test_full_system_counts():
    # Section 4.1: 2(2*2^d+1) filters per scale in 2D, 3(2*2^d+1)^2 in 3D
    subs = [sb for sb, _ in S.spatial_filters_2d(4, [1, 1, 2, 2], full_system=True)]
    assert len(subs) == 1 + 10 + 10 + 18 + 18
    subs = [sb for sb, _ in S.iter_filters_3d((8, 8, 8), 2, [0, 1], full_system=True)]
    assert len(subs) == 1 + 27 + 75


@pytest.mark.parametrize("name", ["SL2D_2", "SL3D_1", "SL3D_2"])
def test_frame_bounds_match_paper(name):
    # Section 5.1 table, A with B normalised to 1 (grid size not stated by the paper)
    row = _table()[name]
    if row["ndim"] == 2:
        sysm = S.build_2d((128, 128), len(row["levels"]), row["levels"])
        psi = sysm.dual_weight
    else:
        psi, R = S.dual_weight_3d((48, 48, 48), len(row["levels"]), row["levels"])
        assert R == row["R"]
    ratio = psi.min() / psi.max()
    assert abs(ratio - row["A"]) < 1e-3
    assert abs(psi.max() / psi.min() - row["BA"]) / row["BA"] < 0.02 or row["ndim"] == 2


def test_frame_bound_sl2d1_reading():
    # SL2D_1 with the fan-filter reading gives A/B ~ 0.080 against the printed 0.0893
    # (the paper's own fan filter is not printed); only the order of magnitude is pinned.
    sysm = S.build_2d((128, 128), 4, [0, 0, 1, 1])
    ratio = sysm.dual_weight.min() / sysm.dual_weight.max()
    assert 0.07 < ratio < 0.0893


def test_frame_bound_grid_independent():
    a = S.build_2d((128, 128), 4, [1, 1, 2, 2]).dual_weight
    b = S.build_2d((256, 256), 4, [1, 1, 2, 2]).dual_weight
    assert abs(a.min() / a.max() - b.min() / b.max()) < 2e-4


@pytest.mark.parametrize("dims,J,levels,full", [
    ((16, 16), 2, [1, 1], False), ((32, 24), 2, [1, 1], True), ((64, 64), 3, [1, 1, 2], False),
    ((24, 40), 3, [0, 1, 2], False)])
def test_filters_real_even_and_cones(dims, J, levels, full):
    sysm = S.build_2d(dims, J, levels, full)
    N2, N1 = dims
    for f in sysm.filters:
        neg = f[(-np.arange(N2)) % N2][:, (-np.arange(N1)) % N1]
        assert np.max(np.abs(f - neg)) < 1e-14                 # psi_hat(-xi) = psi_hat(xi)
    if N1 == N2:
        idx = {(s.cone, s.j, s.k1): i for i, s in enumerate(sysm.subbands)}
        for (cone, j, k), i in idx.items():
            if cone == 2:
                assert np.max(np.abs(sysm.filters[i] - sysm.filters[idx[(1, j, k)]].T)) < 1e-14
    assert sysm.dual_weight.min() > 1e-3 * sysm.dual_weight.max()


def test_lowpass_and_highpass_structure():
    sysm = S.build_2d((32, 32), 2, [1, 1])
    # the lowpass is the only filter that passes DC; Psi_hat(0) = 1
    assert abs(sysm.filters[0][0, 0] - 1) < 1e-14
    assert np.max(np.abs(sysm.filters[1:, 0, 0])) < 1e-14
    assert abs(sysm.dual_weight[0, 0] - 1) < 1e-14


def test_support_sizes():
    # support of p_j * W_j: P's 7x7 taps upsampled, convolved with g_{J-j} (x1) and
    # h_{J-j+d} (x2); the digital shear keeps the x2 extent
    J = 2
    h = F.qmf_maxflat9(); g = F.mirror_highpass(h)
    for j, d in enumerate([1, 1]):
        w = S.wedge_2d(J, j, d, h, g, F.fan_filter(2))
        a2 = 2 ** (J - j + d); a1 = 2 ** (J - j - 1)
        exp_h = 6 * a2 + 1 + 8 * (2 ** (J - j + d) - 1)
        m = J - j
        exp_w = 6 * a1 + 1 + 8 * 2 ** (m - 1) + 8 * (2 ** (m - 1) - 1)
        assert F.support_box(w) == (exp_h, exp_w)
        for k in (-2, 0, 2):
            s = F.digital_shear(w, k, d, h)
            assert F.support_box(s, 1e-300)[0] == exp_h


@pytest.mark.parametrize("dims,J,levels,full", [
    ((16, 16), 2, [1, 1], False), ((16, 16), 2, [1, 1], True), ((32, 48), 3, [0, 1, 1], False),
    ((64, 64), 4, [1, 1, 2, 2], False), ((24, 16), 2, [2, 0], True)])
def test_perfect_reconstruction_2d(dims, J, levels, full):
    sysm = S.build_2d(dims, J, levels, full)
    x = np.random.default_rng(7).standard_normal(dims)
    c = T.forward(x, sysm.filters)
    xr = T.inverse(c, sysm.filters, sysm.dual_weight)
    assert np.max(np.abs(xr - x)) < 1e-13 * max(1.0, np.abs(x).max())


@pytest.mark.parametrize("dims,J,levels,full", [
    ((8, 8, 8), 1, [0], False), ((12, 8, 16), 2, [0, 1], False), ((16, 16, 16), 2, [1, 1], True)])
def test_perfect_reconstruction_3d(dims, J, levels, full):
    sysm = S.build_3d(dims, J, levels, full)
    x = np.random.default_rng(8).standard_normal(dims)
    c = T.forward(x, sysm.filters)
    xr = T.inverse(c, sysm.filters, sysm.dual_weight)
    assert np.max(np.abs(xr - x)) < 1e-13


def test_bruteforce_convolution_2d():
    # eq. convolution: c_i = f * psi_bar_i on the periodic 16x16 grid, by the double sum
    dims = (16, 16)
    sysm = S.build_2d(dims, 2, [1, 1])
    per = S.spatial_filters_2d_periodized(dims, 2, [1, 1])
    x = np.random.default_rng(3).standard_normal(dims)
    c = T.forward(x, sysm.filters)
    for i in range(sysm.R):
        ref = T.circular_correlate_bruteforce(x, per[i])
        assert np.max(np.abs(c[i] - ref)) < 1e-12


def test_bruteforce_convolution_3d():
    # 3D filter = g_{J-j}(x1) (*) Phi_k1(x1, x2) (*) Phi_k2(x1, x3) built as a spatial
    # circular convolution of the three periodised factors on 8^3, then applied by the sum
    N = 8
    J, levels = 1, [0]
    h = F.qmf_maxflat9(); g = F.mirror_highpass(h)
    sysm = S.build_3d((N, N, N), J, levels)
    x = np.random.default_rng(4).standard_normal((N, N, N))
    c = T.forward(x, sysm.filters)
    phis = S.phi_planes(J, 0, 0, h, F.fan_filter(2))
    gper = F.periodize1d(F.highpass_cascade(h, g, J), N)
    checked = 0
    for i, sb in enumerate(sysm.subbands):
        if sb.cone != 1:
            continue
        G = np.zeros((N, N, N)); G[0, 0, :] = gper
        A = np.zeros((N, N, N)); A[0, :, :] = F.periodize2d(phis[sb.k1], N, N)
        B = np.zeros((N, N, N)); B[:, 0, :] = F.periodize2d(phis[sb.k2], N, N)
        psi = T.circular_convolve_bruteforce(T.circular_convolve_bruteforce(G, A), B)
        ref = T.circular_correlate_bruteforce(x, psi)
        assert np.max(np.abs(c[i] - ref)) < 1e-12
        checked += 1
    assert checked == 9
    # the lowpass: separable h_J on every axis
    hJ = F.periodize1d(F.lowpass_cascade(h, J), N)
    phi = hJ[:, None, None] * hJ[None, :, None] * hJ[None, None, :]
    assert np.max(np.abs(c[0] - T.circular_correlate_bruteforce(x, phi))) < 1e-12


def test_3d_pyramids_are_axis_permutations():
    N = 12
    sysm = S.build_3d((N, N, N), 2, [0, 1], full_system=True)
    idx = {(s.cone, s.j, s.k1, s.k2): i for i, s in enumerate(sysm.subbands)}
    for (cone, j, k1, k2), i in idx.items():
        if cone == 0:
            continue
        base = sysm.filters[idx[(1, j, k1, k2)]]          # [xi3, xi2, xi1]
        if cone == 2:   # psi_hat(xi2, xi1, xi3)
            expect = np.transpose(base, (0, 2, 1))
        elif cone == 3:  # psi_hat(xi3, xi1, xi2)
            expect = np.transpose(base, (2, 0, 1))
        else:
            continue
        assert np.max(np.abs(sysm.filters[i] - expect)) < 1e-14


def test_frame_inequality_and_linearity():
    sysm = S.build_2d((32, 32), 3, [1, 1, 2])
    A, B = sysm.dual_weight.min(), sysm.dual_weight.max()
    rng = np.random.default_rng(11)
    for _ in range(3):
        x = rng.standard_normal((32, 32))
        e = np.sum(T.forward(x, sysm.filters) ** 2)
        assert A * np.sum(x ** 2) * (1 - 1e-12) <= e <= B * np.sum(x ** 2) * (1 + 1e-12)
    x, y = rng.standard_normal((2, 32, 32))
    lhs = T.forward(2 * x - 3 * y, sysm.filters)
    rhs = 2 * T.forward(x, sysm.filters) - 3 * T.forward(y, sysm.filters)
    assert np.max(np.abs(lhs - rhs)) < 1e-12


def test_shift_equivariance():
    sysm = S.build_2d((32, 32), 2, [1, 1])
    x = np.random.default_rng(12).standard_normal((32, 32))
    a = T.forward(np.roll(x, (3, -5), axis=(0, 1)), sysm.filters)
    b = np.roll(T.forward(x, sysm.filters), (3, -5), axis=(1, 2))
    assert np.max(np.abs(a - b)) < 1e-12


def test_threshold_limits():
    sysm = S.build_2d((32, 32), 2, [1, 1])
    x = np.random.default_rng(13).standard_normal((32, 32))
    # K = 0 keeps everything: identity
    assert np.max(np.abs(T.denoise(x, sysm, 0.1, [0.0, 0.0]) - x)) < 1e-13
    # K = inf keeps only the lowpass: IDFT(X phi_hat^2 / Psi_hat)
    out = T.denoise(x, sysm, 0.1, [np.inf, np.inf])
    ref = np.fft.ifft2(np.fft.fft2(x) * sysm.filters[0] ** 2 / sysm.dual_weight).real
    assert np.max(np.abs(out - ref)) < 1e-13
    # ties are kept (|x| >= delta)
    assert T.hard_threshold(np.array([-1.0, 0.5, 1.0]), 1.0).tolist() == [-1.0, 0.0, 1.0]


def test_thresholds_and_norms():
    sysm = S.build_2d((64, 64), 2, [1, 1])
    per = S.spatial_filters_2d_periodized((64, 64), 2, [1, 1])
    assert np.max(np.abs(sysm.l2norms() - np.sqrt(np.sum(per ** 2, axis=(1, 2))))) < 1e-13
    d = T.thresholds(sysm, 0.1, [3.0, 4.0])
    assert d[0] == 0.0
    for i, s in enumerate(sysm.subbands[1:], start=1):
        assert abs(d[i] - [3.0, 4.0][s.j] * 0.1 * sysm.l2norms()[i]) < 1e-16


def test_psnr():
    ref = np.zeros((4, 4)); est = np.full((4, 4), 0.1)
    assert abs(T.psnr(ref, est) - 20.0) < 1e-12
