"""Plain CPU FP64 oracle for real-time CCSD propagation (test infrastructure).

This package is TEST INFRASTRUCTURE. Only ``tests/``, ``__graft_entry__.smoke()``
and the ``cpu_baseline`` leg of ``bench.py`` may import it. The HIP library
and its Python binding never import it and share no code with it.

It evaluates, slowly and plainly in spin orbitals with complex128 NumPy
arithmetic:

* the coupled-cluster equations of motion of the paper's Theory section
  (Eq. derivT for the cluster amplitudes, Eq. derivL for the Lambda
  amplitudes) with a field-dressed Fock matrix (the dipole coupling of the
  linear-absorption subsection; Fock matrix "including the external field"
  of the GPU-implementation subsection) -- module ``ccsd``;
* the dipole expectation value (Eq. dipole) through the Lagrangian identity
  -- module ``ccsd``;
* the Gaussian pulse (Eq. field) and the Dirac-delta kick -- module ``field``;
* the explicit Runge-Kutta family (Eqs. rk_y, rk_k; RK4, Eq. rk4truncation;
  Cash-Karp, Eqs. ck-k, ck-y, ck-h, ck-h-final, trial and adaptive
  propagation) -- module ``integrators``;
* the ground state used as the initial condition (Theory, "Propagation of
  the RT-CC equations") -- module ``ground``;
* a brute-force determinant-space evaluation of the same definitions, used
  only to pin the factorised equations -- module ``bruteforce``.

The absorption-spectrum readout of a dipole trajectory is host-side analysis of
the library's output, not part of the propagation, and lives in the package
(``paper_2205_05175_amd.spectrum``); it is pinned on analytic signals.

Closed-shell variables (used at the boundary) map to spin orbitals as
``t_i^a = t_{i alpha}^{a alpha}`` and ``t_ij^ab = t_{i alpha j beta}^{a alpha b beta}``;
Lambda uses the same map (module ``spinorb``).
"""
