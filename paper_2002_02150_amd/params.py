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


def chirp_duration(m1_msun: float, m2_msun: float, f_star: float) -> float:
    """Time in seconds from the instant the signal's frequency crosses f_star
    to coalescence in the restricted-2PN chirp-time family (Sec. II.B):
    tau0 + tau1 - tau1.5 + tau2."""
    m = (m1_msun + m2_msun) * GM_SUN_S
    eta = m1_msun * m2_msun / (m1_msun + m2_msun) ** 2
    u = math.pi * m * f_star
    tau0, tau15 = chirp_times(m1_msun, m2_msun, f_star)
    tau1 = 5.0 / (192.0 * math.pi * f_star) / u / eta * (743.0 / 336.0 + 11.0 * eta / 4.0)
    tau2 = 5.0 / (128.0 * math.pi * f_star) * u ** (-1.0 / 3.0) / eta * (
        3058673.0 / 1016064.0 + 5429.0 * eta / 1008.0 + 617.0 * eta * eta / 144.0)
    return tau0 + tau1 - tau15 + tau2
