"""FP64 CPU oracle for the state-vector simulator (test infrastructure only).

This package is the checker, not the product. Only the test suite, the smoke
check and the CPU baseline leg of the benchmark may import it; the library in
`paper_2304_14969_amd` never does, and this package imports nothing from it.

Modules
-------
dense   exact Schroedinger-picture simulation of a 2^n complex128 ket, gate by
        gate (Sec. II; QFT of Eqs. qft/dft and the circuit of H and controlled
        phases described after them).
factor  the approximate mode of Sec. III: factorized ket, one-qubit Schmidt
        test via the Bloch vector, SDRP rounding (Eq. sdrp) and the fidelity
        model of Eq. fid_model.
mlp     FP64 forward/backward of the separability-proposal network.

Every function states the passage it follows. Readings of passages that are
ambiguous or garbled are listed where they are used.
"""
