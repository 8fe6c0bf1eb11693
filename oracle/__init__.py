"""Plain CPU FP64 oracle for the scalar-induced gravitational-wave spectrum on
a periodic lattice (arXiv 2605.27231).

TEST INFRASTRUCTURE ONLY.  Nothing in the product (the HIP library and its
Python binding) may import, call, link or execute anything in this package.
It is used by ``tests/``, by ``__graft_entry__.smoke()`` (to check one small
GPU invocation) and by the ``cpu_baseline`` leg of ``bench.py``.

The oracle follows the paper step by step, in FP64, with NumPy/SciPy library
primitives (FFT, symmetric eigensolver, quadrature) as its only building
blocks.  It shares no code with the GPU path; the two meet only in the seeded
input recipes of the ``workloads`` package, which hold no arithmetic of the
method.

Modules
-------
kernels        closed-form time-integral kernels I_s, I_c (Eq. kernels) and the
               radiation-era transfer function they come from (Sec. II)
decomposition  u-grid, kernel matrix and eigen-decomposition (Sec. V)
rng            Philox4x64-10 counter-based generator and its normal deviates
lattice        mode grids and the continuum Fourier convention on the lattice
field          Gaussian realisation, non-Gaussian maps, Phi-hat (Sec. VI)
spectrum       per-target convolution engine, TT projection, shell average,
               Omega_GW (Sec. III, IV)
bruteforce     direct O(N^6) mode sums (Eq. naive_A / naive_B)
semianalytic   Gaussian semi-analytic Omega_GW (Eq. semi_anal)

Parity status: every function is pinned by a ``-m "not gpu"`` test against
a value or property fixed by the paper or by mathematics (see the pin table
in each test module's docstring); none is "parity unpinned".
"""
