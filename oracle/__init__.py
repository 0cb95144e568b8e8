"""FP64 CPU oracle of one Model Tensor Planning replan.

TEST INFRASTRUCTURE ONLY.  This package is the plain, slow reference that the
GPU path is checked against.  Only the test-suite, the smoke check and the
CPU-baseline leg of the benchmark may import it; the product library never
does, and it shares no code with the HIP path.

Modules follow the paper's structure:
  philox     counter-based random numbers (Philox4x32-10, Salmon et al. 2011)
  sampling   random multipartite graph (Def. 1) and path sampling (Alg. 1)
  interp     B-spline (Eq. 3-4, Def. 2) and Akima (Eq. 5-7, Def. 3) interpolation
  dynamics   analytic models f(x,u) and the per-step cost (Eq. 1)
  planner    candidate stack, rollout, top-E, softmax refit (Alg. 2)
"""
