"""MI355X-native EQ-hyperreduced implicit-feature-tracking assembly.

The compute path is ``libift.so`` (HIP, gfx950), reached through the C ABI
of ``include/ift.h``; ``paper_2305_15661_amd.ift`` is its thin binding.
"""
from .ift import Problem, ROM, IftError, hdm_assemble, eq_assemble_residual, eq_assemble_jacobian, \
    rom_gauss_newton_step  # noqa: F401
