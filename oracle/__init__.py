"""Plain FP64 CPU oracle for the enhanced local interpolated bounce-back (ELIBB)
lattice-Boltzmann step of Marson, Thorimbert, Latt & Chopard, "Enhanced
single-node boundary condition for the Lattice Boltzmann Method" (arXiv 2009.04604).

TEST INFRASTRUCTURE ONLY.  Nothing in the product path (the HIP library, its
Python binding) may import, call or link anything in this package; only the
test-suite, the smoke check and the CPU-baseline leg of the benchmark use it.
It shares no code, table or constant generator with the HIP path.

Every function is a slow, direct transcription of the paper's definitions (or of
the textbook definition where the paper relies on one) in float64 NumPy, with no
blocking, fusion or reordering beyond what the definition states:

* ``lattice``   velocity sets and weights (Sec. II.A, c_s^2 = 1/3)
* ``boundary``  the signed link coordinate s, Lagrange coefficients and the
                ELIBB wall/nodal populations (Sec. II.C-E)
* ``geometry``  fluid classification and cut links with exact intersections
* ``solver``    collide (BGK, eq. LB-BGK / Eq2ndOrder, Guo forcing) + stream +
                boundary reconstruction, one full time step
* ``analytic``  closed-form reference flows (Sec. III.A, III.B)
* ``metrics``   rRSE (eq. rRMSE) and related error norms

Parity status per function is recorded in each module header.  Functions pinned
by a test against values the paper or mathematics fixes are marked "pinned";
those with no independent pin are marked "parity unpinned".
"""
