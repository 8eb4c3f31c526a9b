"""CPU oracle for the runtime DAG scheduler and its task kernels.

TEST INFRASTRUCTURE ONLY.  Nothing on the product path may import, call or
execute anything in this package: only ``tests/``, ``__graft_entry__.smoke()``
and the ``cpu_baseline`` leg of ``bench.py`` use it.  It shares no code with
the HIP path (no kernels, headers, helpers, tables or constants); the only
thing both sides consume is the seeded input generator module, which holds
none of the method's arithmetic.

Contents
--------
``dag``    brute-force dependency DAG (pairwise conflict checks), retirement at
           host accesses, and a replay of the stream-assignment policy with a
           brute-force happens-before search for the event waits
           (paper Sec. IV-A, IV-B, IV-C).
``tasks``  plain fp64 reference math of every task kernel the workloads use
           (paper Sec. V-B benchmark descriptions, with the readings listed in
           the design notes where the paper is silent).
``run``    executes a program strictly in program order on the CPU.

Pins: ``tests/test_oracle_*.py`` check every function against values fixed by
the paper's worked DAG cases, closed forms, invariants, library routines and
brute force on tiny inputs.  A function without such a pin says
"parity unpinned" in its docstring.
"""
