"""Seeded synthetic inputs shared by the oracle-side tests and the GPU path.

This package builds AMR hierarchies (oct lists per level) and samples scalar
fields (density, radiative energy, temperature) at cell centres.  It holds none
of the solver's arithmetic: no diffusivity, no face coefficients, no
restriction, no linear algebra.  Every generator is deterministic from its
seed.
"""
from .hierarchy import (  # noqa: F401
    Hierarchy, uniform_hierarchy, centred_box_hierarchy, random_balanced_hierarchy,
    budgeted_hierarchy, cell_coords_of_octs, is_balanced,
)
from .fields import (  # noqa: F401
    PowerLawField, gaussian_pulse, cell_centres,
)
from .configs import (  # noqa: F401
    Problem, config_heat_gaussian, config_fld_lognormal, config_tiny, config_uniform, patch_batch,
)
