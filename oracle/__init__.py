"""CPU oracle of the XDG multigrid solve -- TEST INFRASTRUCTURE ONLY.

A plain, slow, FP64 implementation of what the hot path computes, written from
the paper's definitions.  It exists to check the GPU library: only the test
suite, the entry point's smoke check and the benchmark's CPU-baseline leg may
import it.  It shares no code with the HIP path (no kernels, headers, helpers
or pre/post-processing); both consume the same seeded problems from
`xdg_inputs`, which applies none of the solver's arithmetic.

`mg_omp` is the same solve as `mg` written as plain C++17/OpenMP loops
(mg_omp.cpp, compiled by the package's build step): the timed CPU baseline of
the benchmark, pinned against `mg` and a dense direct solve.

Parity status of every function is listed in its docstring; all solver
functions are pinned by tests under tests/ (dense direct solves, closed forms,
operator identities), none is "parity unpinned" except where stated.
"""
