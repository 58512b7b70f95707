"""MI355X (gfx950) library for linearised-coordinate (LCO) sparse tensors.

Thin Python binding of the C-ABI declared in ``include/lco.h`` (argument
marshalling only: every step of construction, permutation, contraction and addition runs
in the HIP kernels of ``liblco.so``).  PyTorch supplies device memory (through
the caching allocator, bridged by callbacks) and streams.

Functions keep the C names: ``lco_ctx_create``, ``lco_create``,
``lco_permute``, ``lco_contract``, ``lco_add``, ``lco_plan_info`` ... .  See
``paper_1802_02619_amd._lib`` for the argument conventions.
"""
from ._lib import *  # noqa: F401,F403
from ._lib import __all__  # noqa: F401
