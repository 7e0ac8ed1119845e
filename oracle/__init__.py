"""FP64 CPU oracle for the particle-hole polarization-propagator window solve.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or
execute anything in this package: only ``tests/``, ``__graft_entry__.smoke()``
and the ``cpu_baseline`` leg of ``bench.py`` use it, to check the HIP library
against the paper and to time a CPU reference beside it.  The oracle shares no
code with the HIP path; both sides only share the seeded input generator in
``synth/``, which holds none of the method's arithmetic.

Modules
-------
dense      spin-adapted (closed-shell singlet) dense assembly of A, B, S at
           orders 0, 1, 2 and the matrix M, metric Sigma (plain definitions,
           FP64, einsum/matmul only)
spinorb    the same matrices in a general spin-orbital basis, plus the singlet
           projection that links the two routes
fockspace  brute-force Fock-space evaluator: builds H_N, W_N and the MP2 first-
           order wavefunction as explicit matrices over Slater determinants and
           evaluates the defining expectation values of S, A and B directly
pencil     all eigenpairs of the pencil M z = omega Sigma z, window selection
           and dipole oscillator strengths
folded     the paper's interior solver on the CPU: inverse Krylov basis from
           weighted-Jacobi steps with the folded Rayleigh quotient, folded and
           pencil Rayleigh-Ritz, residual-driven restarts (dense matvecs)
columns    exact single columns of M (and of its parts) at any size, for
           sampled parity at sizes where dense assembly is impossible
"""
