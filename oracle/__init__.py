"""CPU FP64 oracle — TEST INFRASTRUCTURE ONLY.

This package is the slow, plainly written reference that the GPU path is checked
against.  Only the test-suite, ``__graft_entry__.smoke()`` and the CPU-baseline
leg of ``bench.py`` may import it; the product library never calls it and has
no CPU fallback.  It shares no code with the GPU path: the only common module
is ``workloads`` (seeded problem descriptions, no solver arithmetic).

Contents
  fem        Q1 (8-node) and Q2 (27-node) hexahedral element routines:
             isotropic linear elasticity and the Holzapfel-Gasser-Ogden model
             with an element-condensed P0 pressure (paper sections 2 and 3),
             follower pressure on 4- and 9-node faces.
  monolithic the plain definition of what FETI computes: global assembly,
             Dirichlet elimination and a sparse direct FP64 solve (section 4
             states FETI as an exact reformulation of this system).
  feti_ref   a CPU reference of the classical and all-floating FETI algebra
             (section 4: tearing, generalised inverses, dual problem,
             projection, preconditioned CG, recovery) used to pin iteration
             counts, condition estimates and dual invariants.
"""
