"""Plain FP64 CPU oracle for LT-AC G0W0 -- TEST INFRASTRUCTURE ONLY.

This package is the slow, obviously-correct reference the GPU path is checked
against.  Only the test suite, the package smoke check and the CPU-baseline
leg of the benchmark may import it; the product path never does.  It shares
no code with the HIP library and does not import it.

Modules (each function cites the passage of Toelle, Niemeyer & Neugebauer,
"Accelerating Analytic-Continuation GW Calculations with a Laplace
Transformation and Natural Auxiliary Functions", that it follows):

* ``grids``   modified Gauss-Legendre frequency grid (Sec. 2, Eq. 7 and
              Sec. 3) and the minimax Laplace grid (Eq. 9, Sec. 3).
* ``naf``     natural auxiliary functions (Eqs. 11-13).
* ``rpa``     sum-over-states and Laplace-transformed polarizability
              (Eqs. 3, 8-10), screening and W_nm (Eq. 2).
* ``sigma``   correlation self-energy on the imaginary axis (Eq. 7).
* ``pade``    Thiele continued-fraction Pade continuation and the
              quasiparticle fixed point (Sec. 2 and Sec. 3).
* ``casida``  brute-force real-axis G0W0 from RPA excitations (the
              "analytic RI" reference of Sec. 4), tiny systems only.
* ``g0w0``    the whole chain.
* ``evgw``    eigenvalue-self-consistent GW on top of it (Sec. 3, Table 3).

Every function is pinned by tests against closed forms, invariants and brute
force; none is marked "parity unpinned".
"""
