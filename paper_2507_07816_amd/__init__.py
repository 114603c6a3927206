"""MI355X-native template-bank evaluation of the long-transient GW detection statistic.

The search step of Merou, Tenorio and Sintes (long-transient gravitational
waves from newborn neutron stars): for every template (f0, tau, n, sky) the
msMagnetar frequency track (Eq. 1), Doppler-shifted (Eq. 2), selects one bin
per segment of a normalised-power spectrogram; the weighted power and the
number count along it are summed (Sec. 2) and ranked by critical ratio
(Eq. 4).  All of it runs in hand-written HIP kernels for gfx950 behind the C
ABI in include/ltgw.h; ``ltgw`` is its ctypes binding.
"""
from . import ltgw  # noqa: F401
from .ltgw import Context, LtgwError  # noqa: F401
