"""MI355X-native resonant-line (Lyman-alpha) Monte Carlo transport.

The hot path (emission, cell march with the Voigt cross-section in the gas
frame, resonant and dust scattering, peeling off, escape binning) runs in the
HIP kernels of ``libthor.so`` behind the C ABI of ``include/thor.h``; this
package only binds it (``thor``) and builds it (``build``).
"""
from . import thor  # noqa: F401
from .thor import Transport, run  # noqa: F401
