"""ORACLE -- test infrastructure, not part of the product.

A plain, slow, obviously correct CPU implementation of what the MBE-FCI hot
path computes, written from the paper (Eriksen & Gauss, "Many-Body Expanded
Full Configuration Interaction. II. Strongly Correlated Regime"):

* ``fci``  -- the energy of one CASCI problem (Sec. 2: the energy of the
  composite space of the reference space and a tuple of expansion orbitals,
  all other occupied orbitals frozen) as the lowest eigenvalue of the
  Slater-Condon Hamiltonian over full-orbital-space determinants (``sc.c``);
  dense ``numpy.linalg.eigvalsh`` on small spaces, ARPACK Lanczos
  (``scipy.sparse.linalg.eigsh``) on a matrix-free product above that.
* ``mbe``  -- the increment recursion of Eq. 3 over orbital tuples that are
  supersets of the reference space [Pi] (Eq. 1-3), the screening rule and the
  order sums.
* ``spin`` -- total spin <S^2> of CAS vectors from S_+ on full-space
  determinants, and the lowest CASCI state of a given total spin.
* ``rdm``  -- one- and two-particle density matrices by explicit operator
  action, the adjoint weights of the increment recursion and the gradient of
  the summed MBE energy with respect to h_pq and (pq|rs).
* ``casscf`` -- CASSCF orbitals of the reference space (the expansion
  reference of Sec. 2): BFGS over the non-redundant rotations with the exact
  gradient, then the canonical orbitals, and the integrals in them.
* ``base``  -- base-model energies of tuples (the expansion of eps - eps_base
  of MBE-FCI-b): second-order Rayleigh-Schroedinger energies of the tuple's
  reference determinant, by brute force over the CAS determinants.
* ``sym``   -- CASCI energies of a given spatial symmetry (Abelian irrep
  labels): the lowest eigenvalue on the determinants of the target irrep.
* ``hf``    -- restricted closed-shell Hartree-Fock orbitals (the paper's
  default expansion orbitals and the reference of its CCSD(T) base), by
  energy descent over the occupied-virtual rotations, and the problem in them.
* ``cc``    -- coupled-cluster base energies (the paper's CCSD(T) base): CCSD
  as the projected similarity-transformed equations on the CAS determinants,
  the (T) correction from the triply excited determinants.

Only ``tests/``, the smoke check of ``__graft_entry__`` and the
``cpu_baseline`` leg of ``bench.py`` may import this package.  It shares no
code with the HIP path; the only common module is ``synth`` (seeded inputs).

Parity unpinned: the screening constants and rule (``mbe.screen_threshold`` and
the child-generation rule) are a reading, since the paper only names the
screening threshold a; they are pinned only by agreement between the two
implementations.
"""
from . import fci, mbe, rdm  # noqa: F401
