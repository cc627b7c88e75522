"""MI355X-native split-step Crank-Nicolson stepper for the spin-1
spin-orbit- and Rabi-coupled Gross-Pitaevskii equations (arXiv:2009.13507).

The kernels live in libssgp.so (HIP, gfx950) behind the C ABI of
include/ssgp.h; ``api`` is the thin Python layer over it and ``autograd`` the
checkpointed real-time adjoint.  ``workloads`` builds seeded inputs and trial
states; ``outputs`` turns a state copied to the host into densities, radial
densities and phases.
Importing this package does not load the library; the first Grid does, and
fails loudly if it has not been built.
"""
__all__ = ["api", "workloads", "outputs", "build"]
