"""Physical constants used by the oracle (SI units).

The paper writes the gyromagnetic ratio as gamma in Eq. 1 and Eq. 6 without a
value.  Eq. 6 only yields a field in A/m when gamma carries units of
m/(A s), i.e. gamma0 = mu0 * gamma_LL with gamma_LL the electron
gyromagnetic ratio in rad/(s T).  That reading is used here.
"""
import math

MU0 = 4.0e-7 * math.pi          # T m / A (vacuum permeability)
GAMMA_LL = 1.7595e11            # rad / (s T)
GAMMA0 = MU0 * GAMMA_LL         # m / (A s), the gamma of Eq. 1 and Eq. 6
KB = 1.380649e-23               # J / K, Boltzmann constant (Eq. 6)
MU_B = 9.2740100783e-24         # J / T, Bohr magneton (Eq. 8)
E_CHARGE = 1.602176634e-19      # C, elementary charge (Eq. 8)
