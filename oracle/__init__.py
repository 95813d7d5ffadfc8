"""CPU FP64 oracle for charge-conserving, time-integrator-agnostic FE-PIC.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call, link or run
anything in this package: only the tests, the smoke check and the benchmark's CPU-baseline
leg use it.  It shares no code, headers, tables or constants with the HIP library; the two
meet only at the seeded inputs produced by ``paper_2102_06248_amd.inputs``.

Everything is computed in float64 with plain loops (the per-particle work lives in
``particles.c``, compiled with gcc) or plain numpy/scipy calls, in the order the paper
states the method:

* ``mesh``        tetrahedral mesh, canonical numbering, incidence matrices (Sec. II-A)
* ``fem``         Whitney 0/1/2 forms and the Hodge / curl-curl matrices (Sec. II-A)
* ``particles``   relativistic Boris push, straight-line path through the tets split at
                  every face, Whitney-1 path integral of the current (Sec. III-B/III-C,
                  Alg. 1, eqs. (chargeDef)-(G))
* ``newmark``     Newmark-beta 3-level update of the wave equation with the
                  time-integrated current as source, Jacobi-PCG, Faraday (Sec. II-B, III-A)
* ``auxspace``    nodal auxiliary-space preconditioner for the Newmark system and PCG
                  with it (the paper leaves the solver open; Hiptmair and Xu 2007)
* ``diagnostics`` nodal charge, continuity and Gauss residuals (Sec. III-A)
* ``pic``         one whole PIC step in the paper's cycle order (Sec. II-A)
* ``mlp``         the per-edge warm-start network, forward/backward/Adam in float64

Where the paper is silent or garbled, each module states the reading it takes.
"""
