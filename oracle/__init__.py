"""FP64 CPU oracle of the PXST reconstruction loop -- TEST INFRASTRUCTURE ONLY.

Nothing in the product path may import this package: only the tests, the smoke
check of the entry module and the CPU-baseline leg of the benchmark use it.  It is
a plain NumPy restatement of the paper's steps (Sec. 2.2.1-2.2.4 and Sec. 4) and
shares no code with the HIP library.
"""
from .pxst_oracle import (  # noqa: F401
    bilinear_weights,
    bilinear_gather,
    bilinear_splat,
    round_half_up,
    update_reference,
    update_pixel_map,
    update_pixel_map_fractional,
    split_half_pixel_maps,
    linear_map,
    reference_contrast,
    defocus_sweep,
    quadratic_refine,
    update_translations,
    pixel_variance,
    calc_error,
    solve,
)
