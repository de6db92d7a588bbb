"""Restricted Hartree-Fock orbitals (mbefci_hf) against the oracle
(oracle/hf.py), and what uses them: the expansion in HF orbitals and the
CCSD(T) base model, whose (T) needs the canonical HF orbitals.

Tolerances: both sides converge the orbital gradient to 1e-10; the energy is
stationary (agreement to 1e-10), the orbitals follow to about 1e-10 / 0.05
(the smallest Hessian estimate), the tuple energies, not stationary in the
orbitals, to a few 1e-9 (bound 1e-8)."""
import numpy as np
import pytest

import synth
from oracle import cc, fci, hf, mbe

torch = pytest.importorskip("torch")
import paper_1905_02786_amd as M  # noqa: E402

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ws():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return M.workspace(2 << 30)


PROBLEMS = {
    "s0": lambda: synth.small_problem(8, 3, 3, [2, 3], nvec=6, seed=0, vec_std=0.15, offdiag_std=0.1),
    "s5": lambda: synth.small_problem(8, 3, 3, [2, 3], nvec=6, seed=5, vec_std=0.15, offdiag_std=0.1),
    "frozen": lambda: synth.small_problem(7, 3, 3, [2, 3], nfrozen=1, nvec=5, seed=4, offdiag_std=0.1, e_const=0.3),
    "hubbard8": lambda: synth.config_hubbard(4.0, nsite=8),
}


@pytest.mark.parametrize("name", list(PROBLEMS))
def test_hf_orbitals_match_oracle(ws, name):
    P = PROBLEMS[name]()
    e_ref, C_ref, eps = hf.rhf(P)
    ctx = M.Context.from_problem(P, device=0)
    out = ctx.hf(ws)
    print(f"{name}: E_HF {out['energy']:.12f} (oracle {e_ref:.12f}), {out['iterations']} steps", flush=True)
    assert abs(out["energy"] - e_ref) <= 1e-10
    U = out["U"]
    assert np.abs(U.T @ U - np.eye(P.norb)).max() <= 1e-12
    assert np.min(np.abs(np.diff(eps[:P.nalpha]))) > 1e-6 and np.min(np.abs(np.diff(eps[P.nalpha:]))) > 1e-6
    sg = np.sign(np.sum(U * C_ref, axis=0))
    assert np.abs(U * sg - C_ref).max() <= 1e-6
    h, eri, c = ctx.hamiltonian()
    Q = hf.transform(P, C_ref)
    D = np.diag(sg)
    assert np.abs(D @ h @ D - Q.h).max() <= 1e-7
    # the Fock matrix of the aufbau determinant is diagonal in the new orbitals
    fa, _ = cc.fock_matrix(replace_h(P, h, eri), list(range(P.nalpha)), list(range(P.nbeta)))
    assert np.abs(fa - np.diag(np.diag(fa))).max() <= 1e-9


def replace_h(P, h, eri):
    from dataclasses import replace
    return replace(P, h=h, eri=eri)


def test_expansion_in_hf_orbitals_matches_oracle(ws):
    """The full-order MBE in the HF orbitals: every tuple energy against the
    oracle's CASCI in its own HF orbitals, the total against the oracle's and
    against frozen-core FCI in those orbitals (the frozen orbital is now the
    lowest HF orbital, so the original frozen-core FCI differs)."""
    P = PROBLEMS["frozen"]()
    _, Q, C = hf.hf_problem(P)
    ctx = M.Context.from_problem(P, device=0)
    ctx.hf(ws)
    res = ctx.run(ws)
    ref = mbe.run(Q)
    worst = 0.0
    for o, ro in zip(res.orders, ref.orders):
        assert [tuple(int(x) for x in t) for t in o.tuples] == [tuple(t) for t in ro.tuples] or o.k == 0
        worst = max(worst, float(np.abs(o.eps - np.asarray(ro.eps)).max()))
    print(f"max |d eps| {worst:.1e}")
    assert worst <= 1e-8
    assert abs(res.total - ref.total) <= 1e-8
    assert abs(res.total - fci.fci_energy(Q)) <= 1e-8


def test_ccsd_t_base_after_hf(ws):
    """HF orbitals make (T) applicable: the CCSD(T) base energies of every
    tuple up to order 2 against the oracle's in its HF orbitals, and the
    base-model expansion's full order equals FCI."""
    P = PROBLEMS["s5"]()
    _, Q, _ = hf.hf_problem(P)
    ctx = M.Context.from_problem(P, device=0, base_model=3)
    ctx.hf(ws)
    import itertools
    X = P.expansion_space()
    worst = 0.0
    for k in (0, 1, 2):
        tl = list(itertools.combinations(X, k)) if k else [()]
        got = ctx.tuple_base(k, tl, ws)
        ref = np.array([cc.base_energy(Q, S, triples=True) for S in tl])
        worst = max(worst, float(np.abs(got - ref).max()))
    print(f"max |d eps_base| {worst:.1e}")
    assert worst <= 1e-8
    res = ctx.run(ws)
    assert abs(res.total - fci.fci_energy(P)) <= 1e-8


def test_open_shell_is_refused(ws):
    P = synth.small_problem(8, 4, 2, [2, 3], nfrozen=1, nvec=6, seed=3)
    with pytest.raises(M.MBEFCIError, match="closed shell"):
        M.Context.from_problem(P, device=0).hf(ws)
