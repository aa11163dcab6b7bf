"""Spatial-domain building blocks of the shearlet filter bank (FP64).

TEST INFRASTRUCTURE ONLY (see the package docstring).

Conventions
  * The DTFT is a_hat(xi) = sum_n a(n) exp(-2 pi i n xi), period 1
    (Section 3.1).
  * A 1D filter is (taps, origin): taps[origin + n] = a(n).
  * A 2D filter is (array, (o2, o1)): array[o2 + n2, o1 + n1] = a(n1, n2);
    axis 0 is x2, axis 1 is x1 (x1 is the fastest, "horizontal" axis).
"""
from math import comb, sqrt

import numpy as np


# ---------------------------------------------------------------------------
# 1D quadrature mirror filter pair (Section 5.1) and cascades (eq. lowhigh)
# ---------------------------------------------------------------------------

def qmf_maxflat9():
    """Symmetric maximally flat 9-tap lowpass h_ShearLab (Section 5.1).

    The paper fixes: 9 taps, symmetric, maximally flat, sum h = 1 and a 3 dB
    point at half the Nyquist band.  With H(w) = h0 + 2 sum_{n=1..4} h_n
    cos(n w) the five unknowns h0..h4 follow from the linear conditions
      H(0) = 1,  H(pi) = 0,  H''(0) = 0,  H''''(0) = 0,  H(pi/2) = 1/sqrt(2).
    Returns the 9 taps h(-4..4) (origin 4).
    """
    n = np.arange(1, 5, dtype=np.float64)
    rows = [
        np.concatenate(([1.0], 2.0 * np.ones(4))),                 # H(0)
        np.concatenate(([1.0], 2.0 * (-1.0) ** n)),                 # H(pi)
        np.concatenate(([0.0], n ** 2)),                            # H''(0)
        np.concatenate(([0.0], n ** 4)),                            # H''''(0)
        np.concatenate(([1.0], 2.0 * np.cos(n * np.pi / 2.0))),     # H(pi/2)
    ]
    rhs = np.array([1.0, 0.0, 0.0, 0.0, 1.0 / sqrt(2.0)])
    half = np.linalg.solve(np.array(rows), rhs)                     # h0..h4
    taps = np.concatenate((half[:0:-1], half))
    return taps, 4


def mirror_highpass(h):
    """g(n) = (-1)^n h(n) with n counted from the centre tap (Section 5.1)."""
    taps, o = h
    n = np.arange(len(taps)) - o
    return taps * (-1.0) ** n, o


def upsample1d(f, m):
    """Insert m-1 zeros between taps: the filter of a_hat(m xi)."""
    taps, o = f
    if m == 1:
        return taps.copy(), o
    out = np.zeros((len(taps) - 1) * m + 1)
    out[::m] = taps
    return out, o * m


def conv1d(a, b):
    """Full linear convolution of two 1D filters."""
    return np.convolve(a[0], b[0]), a[1] + b[1]


def delta1d():
    return np.ones(1), 0


def lowpass_cascade(h, j):
    """h_j: Fourier coefficients of prod_{k=0}^{j-1} h_hat(2^k xi)
    (eq. lowhigh); h_0 is the unit impulse."""
    out = delta1d()
    for k in range(j):
        out = conv1d(out, upsample1d(h, 2 ** k))
    return out


def highpass_cascade(h, g, j):
    """g_j: Fourier coefficients of g_hat(2^{j-1} xi) h_hat_{j-1}(xi)
    (eq. lowhigh), j >= 1."""
    if j < 1:
        raise ValueError("g_j is defined for j >= 1")
    return conv1d(upsample1d(g, 2 ** (j - 1)), lowpass_cascade(h, j - 1))


def dtft1d(f, xi):
    """Evaluate a_hat at arbitrary frequencies xi (array) by the defining sum."""
    taps, o = f
    n = np.arange(len(taps)) - o
    return np.exp(-2j * np.pi * np.multiply.outer(np.asarray(xi, dtype=np.float64), n)) @ taps


# ---------------------------------------------------------------------------
# 2D helpers
# ---------------------------------------------------------------------------

def conv2d(a, b):
    """Full linear 2D convolution, computed as a sum of shifted copies of the
    larger operand weighted by the non-zero taps of the smaller one (exact in
    FP64 up to summation order)."""
    (A, (a2, a1)), (B, (b2, b1)) = a, b
    if np.count_nonzero(A) < np.count_nonzero(B):
        (A, (a2, a1)), (B, (b2, b1)) = (B, (b2, b1)), (A, (a2, a1))
    out = np.zeros((A.shape[0] + B.shape[0] - 1, A.shape[1] + B.shape[1] - 1))
    for r, c in zip(*np.nonzero(B)):
        out[r:r + A.shape[0], c:c + A.shape[1]] += B[r, c] * A
    return out, (a2 + b2, a1 + b1)


def upsample2d(f, m1, m2):
    """Filter of a_hat(m1 xi1, m2 xi2): taps moved to (m1 n1, m2 n2)."""
    A, (o2, o1) = f
    out = np.zeros(((A.shape[0] - 1) * m2 + 1, (A.shape[1] - 1) * m1 + 1))
    out[::m2, ::m1] = A
    return out, (o2 * m2, o1 * m1)


def along_x1(f1):
    """Embed a 1D filter as a 2D filter acting along x1."""
    taps, o = f1
    return taps[None, :].copy(), (0, o)


def along_x2(f1):
    """Embed a 1D filter as a 2D filter acting along x2."""
    taps, o = f1
    return taps[:, None].copy(), (o, 0)


def transpose2d(f):
    """Swap the roles of x1 and x2: b(n1, n2) = a(n2, n1)."""
    A, (o2, o1) = f
    return A.T.copy(), (o1, o2)


def flip2d(f):
    """a_bar(n) = a(-n)."""
    A, (o2, o1) = f
    return A[::-1, ::-1].copy(), (A.shape[0] - 1 - o2, A.shape[1] - 1 - o1)


def flip1d(f):
    taps, o = f
    return taps[::-1].copy(), len(taps) - 1 - o


def outer2d(f_x2, f_x1):
    """Separable filter f_x1 (x) f_x2 as a 2D array [x2, x1]."""
    return np.outer(f_x2[0], f_x1[0]), (f_x2[1], f_x1[1])


def support_box(f, tol=0.0):
    """(height, width) of the bounding box of the taps with |a| > tol."""
    A, _ = f
    rows = np.nonzero(np.any(np.abs(A) > tol, axis=1))[0]
    cols = np.nonzero(np.any(np.abs(A) > tol, axis=0))[0]
    return rows[-1] - rows[0] + 1, cols[-1] - cols[0] + 1


# ---------------------------------------------------------------------------
# Fan filter P (eq. nonsep, Section 5.1)
# ---------------------------------------------------------------------------

def halfband_poly(K):
    """Coefficients (ascending powers of x) of Daubechies' half-band
    polynomial D_K(x) = ((1+x)/2)^K sum_{n<K} C(K-1+n, n) ((1-x)/2)^n,
    which satisfies D_K(x) + D_K(-x) = 1."""
    P = np.polynomial.polynomial
    acc = np.zeros(1)
    for n in range(K):
        acc = P.polyadd(acc, comb(K - 1 + n, n) * P.polypow([0.5, -0.5], n))
    return P.polymul(P.polypow([0.5, 0.5], K), acc)


def fan_filter(K=2):
    """Maximally flat 2D fan filter taps as a 2D filter [x2, x1].

    P(eta) = D_K(x(eta)) with x = (cos 2 pi eta2 - cos 2 pi eta1) / 2
    (McClellan transformation of the half-band D_K).  Its passband is the
    cone |eta2| < |eta1| required by (cond2); P + P(swapped) = 1.
    The taps of x are +1/4 at n2 = +-1 and -1/4 at n1 = +-1; powers of x are
    2D self-convolutions.
    """
    xt = np.zeros((3, 3))
    xt[0, 1] = xt[2, 1] = 0.25
    xt[1, 0] = xt[1, 2] = -0.25
    x = (xt, (1, 1))
    coeffs = halfband_poly(K)
    deg = len(coeffs) - 1
    size = 2 * deg + 1
    out = np.zeros((size, size))
    power = (np.ones((1, 1)), (0, 0))
    for m, a in enumerate(coeffs):
        if m > 0:
            power = conv2d(power, x)
        A, (o2, o1) = power
        out[deg - o2:deg - o2 + A.shape[0], deg - o1:deg - o1 + A.shape[1]] += a * A
    return out, (deg, deg)


def dtft2d(f, xi1, xi2):
    """Evaluate a 2D filter's DTFT at frequencies (xi1, xi2) (broadcast)."""
    A, (o2, o1) = f
    xi1 = np.asarray(xi1, dtype=np.float64)
    xi2 = np.asarray(xi2, dtype=np.float64)
    out = np.zeros(np.broadcast(xi1, xi2).shape, dtype=np.complex128)
    for r, c in zip(*np.nonzero(A)):
        out += A[r, c] * np.exp(-2j * np.pi * ((c - o1) * xi1 + (r - o2) * xi2))
    return out


# ---------------------------------------------------------------------------
# Digital shear operator (eqs. dshear1_alpha, dshear2_alpha)
# ---------------------------------------------------------------------------

def shear_interp_filter(h, d):
    """h_d built from sqrt(2) h: the interpolation filter inside S^d.

    With unit-gain h the upsample/convolve/downsample chain would scale by
    2^-d; sqrt(2) per factor makes S^d_0 a near-identity (reading of the
    paper, which leaves the normalisation open)."""
    taps, o = h
    return lowpass_cascade((sqrt(2.0) * taps, o), d)


def digital_shear(f, k, d, h):
    """S^d_{k / 2^d} applied to a 2D filter f along x1 (eqs. dshear1_alpha
    and dshear2_alpha):
        1. upsample along x1 by 2^d,
        2. convolve along x1 with h_d,
        3. resample by the integer shear S_k: V(n1, n2) = U(n1 + k n2, n2),
        4. convolve along x1 with the flipped h_d,
        5. downsample along x1 by 2^d (keeping the origin)."""
    L = 2 ** d
    hd = shear_interp_filter(h, d)
    U = upsample2d(f, L, 1)
    U = conv2d(U, along_x1(hd))
    A, (o2, o1) = U
    n2 = np.arange(A.shape[0]) - o2
    shift = k * n2                       # V(n1, n2) = U(n1 + shift, n2)
    smax, smin = shift.max(), shift.min()
    V = np.zeros((A.shape[0], A.shape[1] + smax - smin))
    vo1 = o1 + smax
    for r in range(A.shape[0]):
        start = vo1 - o1 - shift[r]
        V[r, start:start + A.shape[1]] = A[r]
    V = conv2d((V, (o2, vo1)), along_x1(flip1d(hd)))
    A, (o2, o1) = V
    c0 = o1 % L
    return A[:, c0::L].copy(), (o2, (o1 - c0) // L)


# ---------------------------------------------------------------------------
# Finite grids
# ---------------------------------------------------------------------------

def periodize2d(f, N2, N1):
    """Sum of all N-periodic translates, placed so that index 0 is n = 0."""
    A, (o2, o1) = f
    out = np.zeros((N2, N1))
    r_idx = (np.arange(A.shape[0]) - o2) % N2
    c_idx = (np.arange(A.shape[1]) - o1) % N1
    np.add.at(out, (r_idx[:, None], c_idx[None, :]), A)
    return out


def periodize1d(f, N):
    taps, o = f
    out = np.zeros(N)
    np.add.at(out, (np.arange(len(taps)) - o) % N, taps)
    return out
