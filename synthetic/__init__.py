"""Seeded synthetic workloads for the FEWHA hot path.

This package holds configuration data (telescope, guide-star asterism,
reconstruction layers, method parameters) and seeded random inputs
(von Karman phase screens with frozen flow, slope noise, random test
vectors).  It contains none of the reconstructor's arithmetic: both the
FP64 CPU oracle and the GPU library take their inputs from here and from
nowhere else.
"""

from .configs import (  # noqa: F401
    ARCSEC,
    CONFIGS,
    get_config,
    truth_of,
)
from .inputs import (  # noqa: F401
    frozen_flow_frames,
    random_vector,
    slope_noise,
    von_karman_screen,
)
