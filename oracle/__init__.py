"""FP64 CPU oracle for two-site ab initio DMRG (test infrastructure only).

This package is the independent reference that the HIP library is checked
against.  It is written from the paper (Chan, Keselman, Nakatani, Li, White,
"Matrix product operators, matrix product states, and ab initio density
matrix renormalization group algorithms") and shares no code with the
library: no kernels, headers, helpers, tables or pre/post-processing.  Only
``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import it; the product path never does.

Modules
  fermions  Jordan-Wigner site operators, the ab initio Hamiltonian on
            determinants (Sec. 2.4, Eq. longrangeh), exact FCI energies.
  mpo       Normal/complementary MPO of that Hamiltonian (Sec. 2.4,
            Eqs. Hdecomp, Sm, norm_complementary, prenormrule), with the
            switch of two-index complementary operators at K/2.
  dmrg      Two-site DMRG sweep with renormalized operators: blocking,
            solving (Davidson), decimation (Sec. 2.1, 2.2, 2.5).
  proj      MPO-free projected-Hamiltonian two-site DMRG for tiny systems.

Parity status of every function is stated in its docstring; functions with
no independent pin say "parity unpinned".
"""
