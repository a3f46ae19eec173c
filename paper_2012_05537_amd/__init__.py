"""MI355X-native semi-Lagrangian lattice Boltzmann hot path (arXiv:2012.05537).

Submodules are imported explicitly: ``inputs`` (seeded synthetic inputs) has
no dependency on the compiled library, ``sllbm`` is the binding of the HIP
C-ABI library, ``adjoint`` the autograd wrapper.
"""
