"""Plain FP64 CPU oracle for the upwind-DG convection operator and its SSP-RK3 substeps.

This package is TEST INFRASTRUCTURE.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import it.  The product path (the HIP library under
``paper_1508_04245_amd/``) never imports, links or calls anything here, and nothing here
imports the product path.  The two share no code: the only module both sides consume is the
seeded input generator ``paper_1508_04245_amd/synth.py``, which holds no arithmetic of the
method (only analytic fields evaluated at caller-given points and seeded noise).

Everything is written for readability, not speed: NumPy FP64, SciPy's Jacobi polynomials and
Gauss-Jacobi rules as library primitives, batched ``einsum`` over elements.

What each module follows in the paper (Lehrenfeld & Schoeberl, arXiv 1508.04245):

* ``refelem``  - the element-wise polynomial space V_h and an L2-orthogonal basis on every
  element (Sec. 2.3, DG space and diagonal mass matrix); Dubiner's orthogonal basis is the one
  the paper names for its facet spaces (Sec. 2.2, realization of projected jumps).
* ``mesh``     - affine simplicial meshes, facets, outward normals (notation of Sec. 1).
* ``dg``       - the upwind trilinear form C_h and the upwind value (Sec. 2.3), the discrete
  operator C^V and the diagonal mass M^V (Sec. 2.3/2.4), and the explicit propagation problem
  ds v + (M^V)^-1 C^V v = 0 (Sec. 3.2, propagation operator) integrated with SSP-RK3.
* ``bruteforce`` - exact rational assembly of the same form on tiny meshes (a pin).
* ``mlp``      - the learned macro-step network in FP64 with manual back-propagation.

Parity pins are listed per function; every function here is pinned by a ``-m "not gpu"`` test
unless its docstring says "parity unpinned".
"""
