"""FP64 CPU oracle for sparse TTV -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, the smoke check in ``__graft_entry__`` and the CPU-baseline
leg of ``bench.py`` may import this package.  The product library
(``paper_2510_01495_amd``) never imports it, and the two share no code.
"""

from .ttv_oracle import (  # noqa: F401
    OracleError,
    abs_sums,
    allbut,
    allbut_abs,
    allbut_products,
    allbut_vjp,
    dense_wanted,
    densify,
    drop_zeros,
    full,
    full_abs,
    full_products,
    mttkrp,
    mttkrp_abs,
    mttkrp_products,
    products,
    regression_grad,
    regression_loss,
    remaining_modes,
    ttv,
    ttv_coords,
    ttv_plain,
    ttv_rows,
    ttv_scaled,
    ttv_entries,
    ttv_vjp,
)
