"""Reference oracle for the DPG multigrid solver (test infrastructure only).

This package is a plain, slow, FP64-complex CPU implementation of what the
GPU library computes, written from the paper (Badger, Henneking, Petrides,
Demkowicz, "Scalable DPG multigrid solver for Helmholtz problems: a study on
convergence", arXiv 2304.01728):

* ``basis1d``   -- 1-D Gauss rules, Legendre and hierarchical H1 shape
                   functions, two-scale (refinement) matrices.
* ``element``   -- element Gram matrix of the adjoint graph test norm (Sec. 2,
                   eq. Gnorm), element matrix of the broken ultraweak form and
                   its load (Sec. 2, the forms b, b-hat, l), by quadrature.
* ``dpg``       -- optimal test product B^H G^-1 B with enriched test space
                   (Sec. 2, first paragraph), static condensation onto traces
                   (Sec. 1.2), global assembly, direct solve, field recovery.
* ``topology``  -- canonical numbering of trace unknowns, macro-grid sets,
                   vertex patches, natural-inclusion prolongation (Sec. 3).
* ``multigrid`` -- hierarchy by Galerkin restriction, additive Schwarz
                   vertex-patch smoother, V-cycle and preconditioned CG on the
                   macro grid (Sec. 3 and the solver parameters of Sec. 4).

Only the test-suite, the smoke check and the CPU-baseline leg of the
benchmark may import this package.  The GPU library never does, and this
package never imports the GPU library.
"""
