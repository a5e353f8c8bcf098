"""Plain, slow FP64 CPU oracle for the dense EFIE method-of-moments path.

TEST INFRASTRUCTURE ONLY.  Only tests/, __graft_entry__.smoke() and the
cpu_baseline leg of bench.py may import anything here; the GPU library never
does, and this package imports nothing from the library (only the seeded input
generators in paper_2606_13482_amd.inputs serve both sides).

Everything here is written from the paper's statement of the problem
(Sec. II: EFIE operator, Green's function, RWG Galerkin matrices eq:matTA and
eq:matTPhi, right-hand side) plus textbook mathematics for what the paper
leaves open (quadrature rule, singular integrals, Krylov solvers, convergence
criteria, Mie series).  Each module states the passage or the published
method it follows.

Modules
  mesh        RWG table (Sec. II, RWG without edge-length normalisation; Sec. VI-A figure)
  quadrature  Radon 7-point rule and collapsed Gauss rules on triangles
  potentials  closed-form integrals of 1/R and (y-x)/R over a triangle
  efie        dense Galerkin EFIE fill, plane-wave RHS, far field / RCS, star matrix
  krylov      LU, restarted GMRES (MGS), CGNR, SCC and RSCC criteria
  sampling    SplitMix64 and Floyd's sampling for the random-sampling criterion
  mie         Mie series of a PEC sphere (check path)
  calderon    barycentric refinement, BC functions, mixed Gram matrix and the
              multiplicative Calderon preconditioner (Andriulli et al. 2008)
"""
