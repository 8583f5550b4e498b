"""Plain, slow, CPU FP64 oracle for the multigrid Poisson solve.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import anything from this package.
The product path (the HIP library and its Python binding) never imports,
links or calls it, and this package imports nothing from the product.

Modules
-------
poisson  periodic-level solve: discrete operator, FFT direct solve, red-black
         Gauss-Seidel, restriction, prolongation, V-cycle, mixed precision.
morton   Morton keys (bit loop), decode, neighbour/parent/child keys,
         brute-force oct-neighbour search.
amr      refined (Dirichlet) levels: ghosts by trilinear interpolation of the
         coarse potential, the level operator, direct/CG solve, and the masked
         father-cell multigrid hierarchy.
cnn      reference 3-D convolution network (circular padding, exact GELU),
         forward and backward, Adam.
"""
