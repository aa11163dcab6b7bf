"""Plain FP64 CPU oracle of the digital shearlet transform (ShearLab 3D,
Kutyniok, Lim, Reisenhofer 2014).

TEST INFRASTRUCTURE ONLY.  Nothing in the product package imports, links or
runs this code; only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may use it.  It shares no code with the
HIP path: the filter bank here is built the way the paper constructs it, in
the spatial domain (1D wavelet cascades, a fan filter, upsampling, the digital
shear operator, periodisation and a DFT), while the library evaluates its own
closed form of the same filters in the frequency domain.

Modules
  filters    1D QMF pair and cascades (Section 5.1, eq. lowhigh), the fan
             filter P (eq. nonsep, Section 5.1), 2D/1D spatial helpers
  system     2D and 3D shearlet filter banks (Section 3.2, 3.3, 3.4, 4.4)
  transform  forward / inverse transform (Algorithms 1 and 2, eq.
             reconstruction), hard thresholding, PSNR, brute-force
             circular convolution
  cnn        learned-shrinkage CNN forward/backward in FP64 with an optional
             BF16 rounding emulation

Readings of points the paper leaves open:
  * h is the symmetric 9-tap maximally flat lowpass fixed by H(0)=1,
    H(1/2)=0, H''(0)=H''''(0)=0 and |H(1/4)|=1/sqrt(2) (3 dB at half band).
  * g(n) = (-1)^n h(n) with n centred on the middle tap.
  * P is the McClellan-mapped maximally flat half-band fan filter
    D_2((cos 2 pi eta2 - cos 2 pi eta1)/2); parity with the toolbox filter
    the paper names is unpinned.
  * The cascade inside the digital shear uses sqrt(2)*h so that S^d_0 is
    close to the identity; W_j and the lowpass use unit-gain h.
  * Filters whose spatial support exceeds the grid are periodised.
  * j0 = 0; cone 2 drops k = +-2^{d_j}; in 3D the lower-indexed pyramid
    keeps every seam filter.
"""

__all__ = ["filters", "system", "transform", "cnn"]
