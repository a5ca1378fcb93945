"""The whole fast aperture-mass path, step by step (oracle).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

shear -> KS inversion (Sec. 1, Sec. 4.5) -> starlet planes (Sec. 3) -> noise
maps from randomised shears and S = M_ap / sigma (Sec. 1) -> peak counts per
scale (Sec. 2.2).
"""

from .ks import ks_invert
from .starlet import starlet_forward
from .noise import noise_sigma, snr_planes
from .peaks import count_peaks_planes


def run_path(g1, g2, J, n_real, seed, threshold=3.0):
    """Return a dict with kappa_E, kappa_B, planes, sigma, snr and peaks."""
    kE, kB = ks_invert(g1, g2)
    planes = starlet_forward(kE, J)
    sigma = noise_sigma(g1, g2, J, n_real, seed)
    snr = snr_planes(planes, sigma)
    peaks = count_peaks_planes(snr, threshold)
    return {"kappa_e": kE, "kappa_b": kB, "planes": planes, "sigma": sigma,
            "snr": snr, "peaks": peaks}
