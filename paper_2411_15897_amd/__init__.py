"""MI355X-native block-acoustic preconditioned elastic Helmholtz solver.

The solver (Yovel & Treister, "A block-acoustic preconditioner for the
elastic Helmholtz equation") runs in hand-written HIP kernels for gfx950
behind the C ABI of include/ehelm.h (libehelm.so).  This package holds the
thin ctypes binding (`solver.ElasticHelmholtz`) and the
`torch.autograd.Function` of the full-waveform-inversion misfit
(`fwi.ElasticMisfit`).
"""
from .solver import ElasticHelmholtz, EhelmError, default_abc_sides  # noqa: F401

__all__ = ["ElasticHelmholtz", "EhelmError", "default_abc_sides"]
