"""Seeded synthetic inputs for sparse tensor-times-vector workloads.

This package only draws random tensors and vectors.  It holds none of the
arithmetic of the TTV method, so both the CPU oracle and the GPU path may use
it as their common source of inputs.
"""

from .workloads import (  # noqa: F401
    COO,
    BatchMember,
    seeds,
    tiny,
    uniform_distinct,
    uniform_iid,
    vector,
    zipf_iid,
    workload_small,
    workload_uniform,
    workload_zipf,
    workload_batch,
    workload_grad,
    workload_paper_sweep,
)
