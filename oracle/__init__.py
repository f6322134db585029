"""CPU reference ("oracle") for the O(N) direct solver of Corona, Martinsson
and Zorin, "An O(N) Direct Solver for Integral Equations on the Plane".

TEST INFRASTRUCTURE ONLY.  Nothing in the library imports, links or calls
this package; only the test-suite, the smoke check and the CPU-baseline leg
of the benchmark do.  It shares no code with the HIP path.

Contents (plain, slow, obviously correct, float64 / complex128):
  nystrom  -- kernel functions, self-cell integrals, dense Nystrom assembly,
              exact matrix-vector products (direct sum and FFT convolution)
  dense    -- dense LU solve of the exact discrete system
  krylov   -- restarted GMRES on the exact matvec, for sizes too large to
              assemble
  rskel    -- the paper's recursive-skeletonisation inverse (Algorithm 1 with
              the boundary-layer skeletons of Sec. 3.1 and proxy interpolation)
              followed by the inverse apply, written in the paper's notation
  hssc     -- the compressed-block (HSS-C) inverse of Sec. 3.3: HSS1D and
              low-rank arithmetic, INTER_LOWRANK, BUILD_Finv / APPLY_Finv,
              BUILD_E (Algorithms 3-5) and the inverse apply (Algorithm 6)
              for boxes above a skeleton size k_cut
"""
