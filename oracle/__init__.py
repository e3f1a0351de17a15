"""FP64 CPU oracle for the corner-transfer (CTMRG) move of Lan & Evenbly,
"Reduced Contraction Costs of Corner-Transfer Methods for PEPS".

TEST INFRASTRUCTURE ONLY.  Nothing on the product path may import, call or
execute anything in this package: only the test suite, the package smoke
check and the benchmark's CPU-baseline leg do.  It shares no code with the
HIP library and imports nothing from it.
"""

from .ctm import (  # noqa: F401
    TAU,
    STANDARD,
    REDUCED,
    REDUCED_ENV,
    double_layer,
    heisenberg_h2,
    truncate,
    init_env,
    rotate_site,
    frame_env,
    unframe_env,
    anchor_standard,
    anchor_reduced,
    anchor_reduced_env,
    reduced_half_network,
    absorb_chain,
    move,
    ctm_iteration,
    corner_spectra,
    bond_energy,
    energy,
    site_rdm,
    expect1,
    staggered_magnetisation,
    row_correlation,
    solve,
    CORNERS,
    ENV_KEYS,
)
