"""CPU oracle: a plain, slow, FP64 (complex128) implementation of the hot path.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import or call it:
only tests/, __graft_entry__.smoke() and bench.py's cpu_baseline leg do.  It
shares no code with the HIP library; its inputs come from the generator module
``fields`` (which contains none of the method's arithmetic).

Every function follows a passage of the paper (arXiv 2505.14399,
"Accelerating multigrid with streaming chiral SVD for Wilson fermions in
lattice QCD") cited in its docstring; where the paper is silent (the Wilson
operator's formula, gamma basis, boundary conditions, smoother, cycle) the
reading is stated beside the code.

Modules
  geometry   lexicographic sites, neighbour/sign tables, aggregates, coarse neighbours
  gamma      chiral gamma basis, chirality projectors
  wilson     Wilson-Dirac D and D^dagger (stencil + dense builder)
  clover     clover leaves, field strength, the clover term and the Wilson-clover operator
  evenodd    even-odd (Schur-complement) preconditioning of the fine operator
  philox     Philox4x32-10 counter RNG and Box-Muller (test-vector guesses)
  krylov     GMRES (smoother, coarse solver), flexible GCR
  icsvd      chiral split, Algorithm 3 (iCSVD) with LAPACK SVD, Algorithm 2, Algorithm 1
  transfer   prolongator P (Eq. 6), R = P^dagger
  coarse     Galerkin coarse operator (Eq. 5) as a 9-block stencil, coarse apply
  coarse_evenodd  even-odd (Schur-complement) form of the coarse stencil on the aggregate colouring
  mg         test-vector smoothing (Eq. 2), setup (Algorithm 4), K-cycle, MG solve
  force      gradient of Re<eta, D^-1 b> w.r.t. b and the gauge links
  level      the next coarser level of a coarse stencil (a third level): coarse test
             vectors, chiral split by sigma3, Algorithm 3, coarse-coarse Galerkin operator,
             three-level K-cycle solve

Parity status: every function is pinned by a CPU test against a closed form,
an invariant, a special case or brute force, except the MG iteration counts
(parity unpinned: the paper prints counts only for ensembles that are not
available).
"""
