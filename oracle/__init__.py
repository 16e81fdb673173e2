"""Plain FP64 CPU oracle for the force-field kernel ridge solve.

TEST INFRASTRUCTURE ONLY.  Only the tests, the package smoke check and the CPU
baseline leg of the benchmark may import this package.  It shares no code with
the HIP library: it is a slow, direct transcription of the definitions in the
paper (and of the kernel the workloads fix), written with numpy/scipy in
float64 so that a reader can check it against the paper by eye.

Modules
  kernel  -- inverse-distance descriptor, its Jacobian, the Matern-5/2 force
             kernel, dense assembly and a per-pair matrix-free product
  solve   -- closed-form Cholesky solve, textbook (preconditioned) CG,
             Nystroem/Woodbury preconditioner
  select  -- counter-based SplitMix64 stream, uniform and weighted sampling,
             incomplete Cholesky (pivoted or in a given order), ridge leverage
             scores (exact and pilot estimate)
  mlp     -- the score-predicting MLP: forward, backward, Adam
  rot     -- rule-of-thumb preconditioner size
  symmetry -- the kernel symmetrized over a group of atom permutations

Parity status of every function is listed in its module docstring.
"""
