"""Physical constants used by the oracle (SI; IAU 2015 nominal solar values).

The paper does not print these; they are the standard values.  The GPU library
carries its own copy, written separately.
"""
import math

C_SI = 299792458.0                       # speed of light [m/s]
GM_SUN = 1.3271244e20                    # nominal solar mass parameter [m^3 s^-2]
MTSUN_S = GM_SUN / C_SI ** 3             # G Msun / c^3 [s]
MPC_M = 3.085677581491367e22             # megaparsec [m]
EULER_GAMMA = 0.57721566490153286060651209008240243
PI = math.pi
