"""FP64 CPU oracle for the Wilson and 2-flavour staggered Wilson CGNR path.

TEST INFRASTRUCTURE ONLY.  This package is a plain, slow, numpy implementation of
what the GPU library computes, written from the paper (Adams, Nogradi, Petrashyk,
Zielinski, "Computational efficiency of staggered Wilson fermions: A first look",
LATTICE 2013) and from the operator definitions it relies on.  Only the tests,
``__graft_entry__.smoke()`` and the benchmark's CPU-baseline leg may import it;
the library never does, and this package imports nothing from the library.
Shared with the GPU side is only ``synth`` (seeded inputs, no method arithmetic).

Modules:

* ``lattice``  -- shifts with fermion boundary signs, staggered phases;
* ``gauge``    -- mean plaquette, gauge transformations, epsilon tuning;
* ``wilson``   -- Wilson Dirac matrix D_W + m and its adjoint (Sec. 2, eq. (2));
* ``staggered_wilson`` -- staggered hopping term, Gamma_55 in three forms,
  D_SW + m and its adjoint (Sec. 2, eq. (2));
* ``solvers``  -- CG on the normal equations (eq. (2)) and Lanczos for the
  condition number (Sec. 3);
* ``freefield`` -- closed-form free-field spectra (Sec. 3, the 8/sqrt(5) limit);
* ``dense``    -- dense matrices of the operators on small lattices;
* ``critical`` -- m_c as the minimiser of the Lanczos lowest eigenvalue;
* ``evenodd``  -- even-odd (Schur complement) preconditioned CG for Wilson
  (footnote to eq. (2), Sec. 3);
* ``evenodd_sw`` and ``study_sw_evenodd`` -- the same block elimination for
  staggered Wilson, with inner solves, to measure its cost;
* ``spectroscopy`` -- the Wilson pion correlator and effective mass (Fig. 1(a));
* ``spectrum`` -- dense eigenvalues of the Dirac matrix and the free staggered
  Wilson spectrum (Fig. 1(c));
* ``overlap``  -- the staggered overlap operator with the staggered Wilson
  kernel (Secs. 1, 2 and 4): exact from the dense sign function, and the
  Chebyshev polynomial approximation of the GPU path.
"""
