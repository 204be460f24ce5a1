"""Seeded synthetic inputs for the jump-SDE proton dose path.

This package holds only input data: material compositions, phantom
geometries, beam and plan descriptions and the placeholder nuclear
tables.  It contains none of the transport arithmetic.  Both the FP64
oracle (``oracle/``) and the HIP path (``paper_2511_03115_amd``) consume
what it produces; neither imports the other.
"""

from .materials import ELEMENTS, material, water, bone, lung  # noqa: F401
from .nuclear import placeholder_nuclear_tables, nuclear_for_phantom, EnergyLattice  # noqa: F401
from .phantoms import (Phantom, water_box, slab_phantom, insert_phantom,  # noqa: F401
                       grf_phantom)
from .beams import Spot, single_spot, plan_spots, patch_spots, with_histories  # noqa: F401
from . import configs  # noqa: F401
