"""Plain FP64 CPU oracle for the tensor jump method (TJM).

TEST INFRASTRUCTURE ONLY.  Nothing in the product package may import, call,
link or execute anything in this directory; only ``tests/``,
``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of ``bench.py`` use
it.  It shares no code with the HIP path: the two meet only in the seeded
input generators of ``tests/inputs.py`` and in the published definition of
the Philox4x32-10 counter-based generator, which each side implements on its
own.

Modules
-------
philox      Philox4x32-10 (Salmon et al., SC'11) and the TJM draw layout.
model       Pauli matrices, the XXX / TFIM Hamiltonians as MPOs and as dense
            Kronecker sums, jump-operator sets, the local dissipators D_l.
lindblad    Exact vectorised Lindblad integration (Eq. Lindblad), L <= 8.
dense_tjm   The TJM schedule on dense state vectors (exact U), and the
            textbook first-order MCWF, L <= 10.
mps_tjm     The TJM on matrix product states, step by step as the paper's
            Sec. "Tensor jump method" describes it: dynamic TDVP with Lanczos
            exponentials, QR/SVD sweeps, dissipative contraction, jump process.

Every floating-point computation is complex128 / float64.
"""
