"""Physical constants in cgs (oracle copy; test infrastructure only).

Lsun follows the FSPS value quoted in Sec. 2.6; the AB zero point is the
3631 Jy flux density of App. E; the FWHM/sigma ratio is eq. (F1).
"""
import math

C_CMS = 2.99792458e10            # speed of light [cm/s]
C_KMS = 2.99792458e5             # speed of light [km/s]
H_PLANCK = 6.62607015e-27        # Planck constant [erg s]
LSUN = 3.839e33                  # solar luminosity [erg/s] (Sec. 2.6)
PC_CM = 3.0856775814913673e18    # parsec [cm]
MPC_CM = 1e6 * PC_CM
MPC_KM = MPC_CM / 1e5
YR_S = 3.15576e7                 # Julian year [s]
FNU_AB = 3.631e-20               # AB zero point [erg/s/cm^2/Hz] (App. E)
ANG_CM = 1e-8                    # Angstrom [cm]
FWHM_PER_SIGMA = 2.0 * math.sqrt(2.0 * math.log(2.0))   # eq. (F1)
LAM_LYMAN = 912.0                # Lyman limit [A] (eq. C1)
LAM_V = 5500.0                   # attenuation reference wavelength [A] (Sec. 2.4)
