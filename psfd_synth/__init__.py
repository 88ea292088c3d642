"""Seeded synthetic inputs for the PSFD solver: workload parameters and mask layouts.

This package holds input data only (grid sizes, optical constants, seeded
binary layouts, seeded random fields).  It contains none of the solver's
arithmetic, so both the plain CPU reference under ``oracle/`` and the HIP
library can take their inputs from it without sharing any computation.
"""

from .configs import (  # noqa: F401
    ML_BILAYERS,
    N_MO,
    N_SI,
    base_config,
    config_c1,
    config_c2,
    config_c3_sizes,
    config_c4,
    config_c5,
    FULL_DOMAIN_NZ,
    FULL_DOMAIN_THETAS_DEG,
    eps_absorber_default,
    ffno_desc,
    ffno_weight_blocks,
    ffno_weights,
    full_domain_config,
    full_domain_stack,
    multilayer_stack,
    nz_total,
)
from .layouts import (  # noqa: F401
    contact_holes,
    curvilinear,
    line_space,
    random_field,
    rect_layout,
    smooth_perturbation,
)
