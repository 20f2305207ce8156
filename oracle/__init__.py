"""CPU oracle for the task-ordering temporal execution model.

TEST INFRASTRUCTURE ONLY.  Nothing on the product path imports, links or runs
anything in this package: only the test-suite, the smoke check and the CPU
baseline leg of the benchmark do.  It shares no code with the HIP library.

Modules
  model      -- the event-driven simulator of Section 4.1 (integer-ns and exact
                rational modes), brute force over all orderings, summaries, and
                the ordering heuristic of Section 5.1 (Algorithm 1).
  cmodel     -- ctypes loader of ``tgo_oracle.c``, a plain C transcription of
                the same integer simulator for large enumerations.
  mlp        -- float64 reference of the surrogate network (forward, loss,
                analytic backward) used to check the GPU training kernels.
  philox     -- the Philox4x32-10 counter-based generator and the ordering
                sampler built on it.
"""
