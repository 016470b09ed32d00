"""MI355X-native D3Q27 chemical-potential free-energy lattice Boltzmann step
(arXiv:2504.03819) behind the C ABI of include/lbfe.h.

Submodules:
  lbfe      ctypes binding of the HIP library (Simulation, Params, constants)
  autograd  torch.autograd.Function over the hand-written adjoint with
            checkpoint-every-K recomputation
  inputs    seeded synthetic initial fields of the benchmark problems
  build     hipcc build of _lib/liblbfe.so
"""
from . import inputs  # noqa: F401
