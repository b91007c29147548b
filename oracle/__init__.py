"""Reference CPU oracle for the elastic-solid lattice Boltzmann scheme (D2Q9, and D3Q19).

TEST INFRASTRUCTURE. Everything under ``oracle/`` exists to check the GPU
library, never to stand in for it: only ``tests/``, the package smoke check and
the CPU-baseline leg of ``bench.py`` may import, call, link or run it. It shares
no code with ``paper_2009_06404_amd`` and imports nothing from it.

* ``lbm_oracle.c`` / :mod:`oracle.stepper` -- the scheme itself (FP64, the
  paper's collide-then-push-stream form of eq. LBGK, Sec. 2 and 6).
* :mod:`oracle.theory` -- von Neumann matrix (Sec. 4), wave speeds (Sec. 2),
  Rayleigh-wave root (Sec. 7).
* :mod:`oracle.spectral` -- the Fourier / Crank-Nicolson reference of App. B.
* ``lbm3d_oracle.c`` / :mod:`oracle.stepper3d` -- the same step on the
  three-dimensional D3Q19 lattice (Sec. 3's regular lattices), FP64, with the
  face rules of Sec. 6 read for a volume.
* :mod:`oracle.filter` -- the high-wavenumber filter of a state (Sec. 4's
  remedy for the instability of nu != 1/4; the form is the library's own).
"""
