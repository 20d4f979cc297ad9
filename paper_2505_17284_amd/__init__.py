"""MI355X-native explicit discrete-ordinates (S_N) finite-volume transport step.

The package computes the explicit S_N transport step of Schotthoefer & Hauck,
"Reference solutions for linear radiation transport: the Hohlraum and Lattice
benchmarks" (arXiv 2505.17284), Sec. 4 (eqs. ``eq_sn_2d``, ``eq_sn_2d_eqn_fv``,
``eq_ODE``), on a uniform 2-D Cartesian grid, with hand-written HIP kernels for
gfx950 behind the C ABI declared in ``include/snrt.h``.

Importing the package loads nothing native. ``inputs`` builds problem
statements (geometry masks, cross-sections, quadrature); ``solver`` drives the
native library through ``_lib``.
"""

__version__ = "0.1.0"

__all__ = ["inputs", "solver", "__version__"]
