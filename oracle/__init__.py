"""Plain FP64 CPU oracle for the Toeplitz MBIR hot path — TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import this package.  The product path (the HIP library and its
Python binding) never imports, calls or links anything here, and nothing here
imports the HIP package: the two share no code.  Inputs common to both come from
the separate ``synth`` package, which holds no arithmetic of the method.

Every function states the passage of the paper (arXiv 2603.28756) it follows.
Where the paper is silent or garbled the reading taken is stated in the
docstring; all readings are collected in the design notes of the repository.

Modules
-------
geometry   pixel/detector coordinates and the polar Fourier sample set (Sec. 2, Eqs. 2-4)
radon      exact non-uniform DFT forward operator A = F^-1 NUFFT2 and its adjoint (Eqs. 3-4)
toeplitz   point-spread function K, its padded spectrum and the Toeplitz product (Sec. 2.1)
prior      qGGMRF potential, value and gradient over 8 or 26 neighbours (Sec. 2, Eq. 5)
fbp        ramp-filtered back-projection initial estimate (Sec. 2.2, Eqs. 12-14)
solver     objective, gradient, Lipschitz constant and FISTA with restart (Sec. 2, Eqs. 5-6, 10-11)
hierarchy  sinogram subsampling, Lanczos-3 prolongation, coarse-to-fine solve (Sec. 2.3)
unet       learned start: U-Net forward, backward, loss and Adam step (Sec. 2.2, 3.2 extension)
"""
from . import geometry, radon, toeplitz, prior, fbp, solver, hierarchy, unet  # noqa: F401
