"""Free-space constants (SI).  Time convention exp(+j w t)."""
import math

C0 = 299792458.0
MU0 = 4.0e-7 * math.pi
EPS0 = 1.0 / (MU0 * C0 * C0)
ETA0 = MU0 * C0


def wavenumber(freq_hz: float) -> float:
    return 2.0 * math.pi * freq_hz / C0
