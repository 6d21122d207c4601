"""Parameter conversions used to set up searches and synthetic signals."""
import math

GM_SUN_S = 4.925490947e-6


def chirp_times(m1_msun: float, m2_msun: float, f_star: float):
    """(tau0, tau1.5) in seconds from component masses (Sec. II.B definitions)."""
    m = (m1_msun + m2_msun) * GM_SUN_S
    eta = m1_msun * m2_msun / (m1_msun + m2_msun) ** 2
    u = math.pi * m * f_star
    return (5.0 / (256.0 * math.pi * f_star) * u ** (-5.0 / 3.0) / eta,
            1.0 / (8.0 * f_star) * u ** (-2.0 / 3.0) / eta)
