"""SI constants used by the oracle (CODATA 2018).  Typed here independently of the HIP
library, which carries its own copy."""

EPS0 = 8.8541878128e-12        # F/m, vacuum permittivity
MU0 = 1.25663706212e-6         # H/m, vacuum permeability
C_LIGHT = 299792458.0          # m/s
Q_E = 1.602176634e-19          # C, elementary charge
M_E = 9.1093837015e-31         # kg, electron mass
