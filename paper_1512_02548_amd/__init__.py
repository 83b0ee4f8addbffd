"""MI355X-native hot path of the stabilised nodal spectral element method for
fully nonlinear potential-flow water waves (Engsig-Karup, Eskilsson & Bigoni,
arXiv:1512.02548).

The numerical work runs in hand-written HIP kernels behind the C ABI declared
in ``include/sem.h`` (shared library ``libsem.so`` built from ``csrc/``).
``paper_1512_02548_amd.lib`` is the thin ctypes binding; importing this package
does not load the library, so the input generators in ``workloads`` can be
used without a GPU.
"""
__all__ = ["lib", "workloads"]
