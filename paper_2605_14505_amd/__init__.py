"""MI355X (gfx950) implementation of the stratified Taylor-Green DDF lattice Boltzmann step.

The compute path is the HIP library ``lib/libstgv.so`` behind the C ABI in
``include/stgv.h``; ``paper_2605_14505_amd.stgv`` is its Python binding.
Build with ``python -m paper_2605_14505_amd.build``.
"""
__all__ = ["build", "stgv"]
