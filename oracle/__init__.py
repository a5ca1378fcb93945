"""FP64 CPU oracle for the fast aperture-mass path of Leonard, Pires & Starck,
"Fast Calculation of the Weak Lensing Aperture Mass Statistic" (arXiv:1204.4293).

TEST INFRASTRUCTURE ONLY.  This package is the plain, slow, obviously correct
reference that the HIP library is checked against.  It is imported only by
``tests/``, by ``__graft_entry__.smoke()`` and by the ``cpu_baseline`` leg of
``bench.py``; the product path (``paper_1204_4293_amd``) never imports, calls or
links it, and it never imports the product path.  It shares no code with the
HIP kernels: no kernels, headers, tables or helpers.

Every routine works on host ``numpy.float64`` arrays (complex128 in Fourier
space), uses loops and ``numpy.roll`` written for clarity, and cites the
passage of the paper it follows.  ``numpy.fft`` is used as the one library
primitive (a plain DFT, no blocking or fusion on top of it).

Conventions shared with the HIP path only through their written definition
(both sides implement them independently):

* maps are square N x N, N a power of two, row-major ``[y][x]``: x is the
  column (fast) index, y the row index; all boundaries are periodic;
* J counts the output planes *including* the smooth plane (Sec. 3: J = j_max+1
  sub-arrays); the planes are ``w_1 .. w_{J-1}, c_{J-1}`` and plane w_j stands
  for the aperture-mass map at theta = 2^j pixels;
* smoothing step j (1-based) uses the B3-spline taps (1,4,6,4,1)/16 at
  dilation 2^(j-1);
* noise phases come from Philox4x64-10 (Salmon et al. 2011) as defined in
  ``oracle.rng``.

Parity status per function (what pins it) is listed in each module's header.
"""

from .filters import (  # noqa: F401
    phi_b3, b3_taps, starlet_U, starlet_Q, starlet_U_from_phi, Q_from_U,
    s98_U, s98_Q, jbj04_U, jbj04_Q, filter_Q_theta, natural_cut,
    FILTER_STARLET, FILTER_S98, FILTER_JBJ04,
)
from .ks import wavenumbers, ks_kernel, ks_invert, dft2_brute  # noqa: F401
from .starlet import (  # noqa: F401
    smooth_step, starlet_forward, starlet_reconstruct, starlet_impulse_response,
    separable_psi_taps, convolve_periodic,
)
from .direct import map_direct, map_direct_at, map_kappa_form_radial  # noqa: F401
from .rng import (  # noqa: F401
    philox4x64_10, phase_uniforms_u32, phase_uniforms, PHILOX_M0, PHILOX_M1,
)
from .noise import (noise_sigma, noise_moments, merge_moments, sigma_from_moments,  # noqa: F401
                    snr_planes, rotate_shear)
from .peaks import count_peaks, count_peaks_planes  # noqa: F401
from .stats import (peak_histogram, peak_histogram_planes, plane_moments,  # noqa: F401
                    plane_moments_stack)
from .pipeline import run_path  # noqa: F401
from .bounded import (  # noqa: F401
    BC_PERIODIC, BC_MIRROR, BC_ZERO, boundary_index, smooth_step_bc, starlet_forward_bc,
    even_extension, ks_invert_padded, noise_sigma_bc, count_peaks_bc,
)
from .masks import mask_shear, count_peaks_masked, count_peaks_masked_planes  # noqa: F401
