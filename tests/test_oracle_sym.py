"""Pins of the symmetry-targeted oracle (oracle/sym.py): the Hubbard dimer's
closed forms per irrep; for a Hamiltonian that respects the labels, the
spectra of the irrep blocks together are the full spectrum (a wrong
determinant label or a missed coupling breaks it); the check of the labels
fails for a Hamiltonian without the symmetry; an empty irrep is an error."""
import numpy as np
import pytest

import synth
from oracle import fci, sym


@pytest.mark.parametrize("U", [2.0, 4.0, 8.0])
def test_hubbard_dimer_closed_forms(U):
    """Two sites, two electrons: bonding (g, label 0) and antibonding (u, 1)
    orbitals.  The lowest g state is the singlet (U - sqrt(U^2 + 16 t^2)) / 2;
    the lowest u state is the M_s = 0 component of the triplet, energy 0."""
    P = synth.config_hubbard(U, nsite=2)
    lab = synth.hubbard_irreps(2)
    assert sym.respects(P, lab)
    assert abs(sym.casci_energy_irrep(P, (), lab, 0) - (U - np.sqrt(U * U + 16.0)) / 2) < 1e-12
    assert abs(sym.casci_energy_irrep(P, (), lab, 1)) < 1e-12


@pytest.mark.parametrize("S", [(), (0, 5), (1, 4, 6)])
def test_irrep_spectra_make_the_full_spectrum(S):
    lab = [0, 1, 2, 3, 0, 1, 2, 3]
    P = synth.symmetric_problem(8, 3, 3, [2, 3], lab, seed=1)
    assert sym.respects(P, lab)
    sp = fci.cas_space(P, S)
    H = fci.hamiltonian_matrix(P, sp)
    full = np.linalg.eigvalsh(H)
    parts = []
    for g in range(4):
        idx = sym.irrep_indices(P, sp, lab, g)
        if idx:
            parts.append(np.linalg.eigvalsh(H[np.ix_(idx, idx)]))
            # no coupling out of the block
            out = [i for i in range(sp.dim) if i not in set(idx)]
            assert np.abs(H[np.ix_(idx, out)]).max(initial=0.0) == 0.0
    assert np.abs(np.sort(np.concatenate(parts)) - full).max() < 1e-10
    lows = [sym.casci_energy_irrep(P, S, lab, g) for g in range(4) if sym.irrep_indices(P, sp, lab, g)]
    assert abs(min(lows) - full[0]) < 1e-10


def test_labels_checked_and_empty_irrep_refused():
    P = synth.small_problem(6, 2, 2, [1, 2], nvec=4, seed=3)
    assert not sym.respects(P, [0, 1, 0, 1, 0, 1])
    Q = synth.config_hubbard(4.0, nsite=2)
    with pytest.raises(ValueError, match="no determinant"):
        sym.casci_energy_irrep(Q, (), synth.hubbard_irreps(2), 3)
