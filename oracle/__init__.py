"""Plain FP64 CPU oracle of the DG + HABC time step (test infrastructure).

This package is test infrastructure, not the product: only the tests, the
smoke check of ``__graft_entry__`` and the CPU-baseline leg of ``bench.py``
may import it.  It shares no code with the HIP library; both read the same
seeded inputs from ``workloads``.

Contents
  reference  nodal reference elements (Section 3.2: Warp & Blend nodes on the
             tetrahedron, triangle and line nodes taken from its faces and
             edges; differentiation and lifting matrices)
  mesh       affine geometry and the four-level connectivity (Section 3.2:
             volume, surface and line meshes and the corners)
  habc       Pade coefficients and the edge/corner compatibility equations
             (Sections 2.1 and 3.1)
  solver     the multidimensional explicit step (Algorithm 1) with the DG
             right-hand sides (Section 3.2) and the five-stage low-storage
             Runge-Kutta scheme; energy
  closure    the small boundary-closure network (forward, gradient), FP64;
             not part of the paper

Every function cites the passage it follows.  Where the paper is silent or
garbled the oracle takes these readings: characteristics carry a factor 1/2,
the 2D and 1D fluxes use Z = rho*c of the boundary cell, and the signs of the
edge and corner systems follow the scalar equations of the procedure.
"""
