"""CPU FP64 oracle for the SP2 / XL-BOMD path — TEST INFRASTRUCTURE ONLY.

This package is the plain, slow, obviously correct reference that the HIP
library is checked against.  Only the test suite, the smoke check and the
CPU-baseline leg of the benchmark may import it; the library itself never
does, and it shares no code, headers, tables or helpers with the library.
Its only common dependency is the seeded input module ``synth``.

Contents (each function cites the passage of Niklasson & Cawkwell,
"Fast method for quantum mechanical molecular dynamics", that it follows):

* ``tb``          orthogonal sp tight-binding Hamiltonian, gamma, pair term
                  (Appendix, SCC-TB subsection: Eqs. DFTB_1, DFTB_2, the
                  gamma / zeta(R) / tail paragraphs);
* ``eig``         LAPACK-free cyclic Jacobi eigensolver (C) + aufbau, the
                  plain definition of theta(mu0 I - H) (orthogonal T_e = 0
                  subsection);
* ``sp2``         second-order spectral projection (SP2) purification,
                  dense and block-thresholded (Linear scaling section);
* ``observables`` Mulliken charges, band energy, potential energy, forces
                  (Eqs. EL_Orth_a-c, HF_POT_2, EtotOrth);
* ``xlbomd``      SCF initialisation and the modified Verlet integration of
                  the auxiliary charges with dissipation (Eq. Verl_n) plus
                  velocity Verlet for the nuclei.

Parity status of every function is recorded in its module header; functions
without an independent pin say "parity unpinned".
"""
