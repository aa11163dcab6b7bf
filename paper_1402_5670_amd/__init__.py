"""MI355X-native digital shearlet transform with compactly supported
shearlets (ShearLab 3D, Kutyniok, Lim, Reisenhofer 2014).

The compute path lives in the HIP shared library ``libshearlet.so`` built
from ``csrc/``; ``binding`` marshals arguments to its C ABI.  Importing this
package does not load the library; ``binding.lib()`` does and raises if it
is missing.
"""
__version__ = "0.1.0"
