"""CPU FP64 oracle for sliced tensor-network amplitudes.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and
the CPU-baseline leg of ``bench.py`` may import or run anything here.  The
engine (``paper_2407_00769_amd``) never imports this package and this package
never imports the engine; both read only the seeded inputs in ``workloads``.

Contents, each a plain and slow definition:
* ``gates``       -- the gate matrices of paper Sec. 2.1.
* ``statevector`` -- FP64 state-vector simulation (paper Sec. 2.2), the plain
                     definition A(x) = <x|U|0^n>; wire projectors give the
                     amplitude of one slice.  Core loop in ``sv.c`` (C/OpenMP).
* ``einsum``      -- naive FP64 pairwise contraction of a labelled network
                     (paper Eq. ``contraction``), with sliced labels fixed
                     by indexing; plus a brute-force sum over assignments.
* ``bruteforce``  -- Kronecker-product unitary of a tiny circuit.
* ``pairwise``    -- one pairwise contraction and single-entry dot products.
* ``metrics``     -- fidelity (paper Eq. ``fidelity``), relative errors,
                     linear XEB and Porter-Thomas distance.
* ``mlp``         -- FP64 forward/backward/Adam of the step-cost MLP.
* ``codec``       -- the low-precision exchange codec (paper Sec. 3.2,
                     Eq. ``quantcal``, Table ``quanttable``, Eq. ``compress``).
* ``postselect``  -- top-k post-selection in a correlated subspace and the
                     linear XEB of the kept samples (paper Sec. 1 and 2.3).
"""
