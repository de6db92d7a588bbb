"""Coupled-cluster base models (options.base_model = 2: CCSD, 3: CCSD(T), the
paper's MBE-FCI-b base of Sec. 4.2.1) against the oracle (oracle/cc.py:
CCSD as the projected similarity-transformed equations on the CAS
determinants, (T) from the triply excited determinants; the library solves
the spin-orbital amplitude equations).  Per-tuple energies within 1e-10
(both sides converge the amplitudes to 1e-11 or below), the expansion of
eps - eps_base within the parity tests' 1e-10 / 1e-9."""
import itertools

import numpy as np
import pytest

import synth
from oracle import cc, fci, mbe

torch = pytest.importorskip("torch")
import paper_1905_02786_amd as M  # noqa: E402

pytestmark = pytest.mark.gpu
TOL = 1e-10


@pytest.fixture(scope="module")
def ws():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return M.workspace(2 << 30)


PROBLEMS = {
    "hubbard8_U2": (lambda: synth.config_hubbard(2.0, nsite=8), 3),
    "hubbard8_U4": (lambda: synth.config_hubbard(4.0, nsite=8), 3),
    "weak": (lambda: synth.config_weak(), 2),
    "open8": (lambda: synth.small_problem(8, 4, 2, [2, 3], nfrozen=1, nvec=6, seed=3, e_const=0.5), 2),
}
CANONICAL = {"hubbard8_U2", "hubbard8_U4"}


@pytest.mark.parametrize("name", list(PROBLEMS))
@pytest.mark.parametrize("model", [2, 3])
def test_tuple_cc_energies_match_oracle(ws, name, model):
    make, kmax = PROBLEMS[name]
    P = make()
    if model == 3 and name not in CANONICAL:
        ctx = M.Context.from_problem(P, device=0, base_model=3)
        with pytest.raises(M.MBEFCIError, match="canonical"):
            ctx.tuple_base(1, [(P.expansion_space()[0],)], ws)
        return
    ctx = M.Context.from_problem(P, device=0, base_model=model)
    X = P.expansion_space()
    worst = 0.0
    for k in range(kmax + 1):
        tl = list(itertools.combinations(X, k)) if k else [()]
        got = ctx.tuple_base(k, tl, ws)
        ref = np.array([cc.base_energy(P, S, triples=model == 3) for S in tl])
        worst = max(worst, float(np.abs(got - ref).max()))
    print(f"{name} model {model}: max |d eps_base| {worst:.1e}", flush=True)
    assert worst <= TOL


def test_full_space_ccsd_t(ws):
    """The whole 8-site space (4900 determinants, 360 amplitudes): the base
    energy that the expansion's total adds."""
    P = synth.config_hubbard(4.0, nsite=8)
    X = tuple(P.expansion_space())
    ctx = M.Context.from_problem(P, device=0, base_model=3)
    got = ctx.tuple_base(len(X), [X], ws)[0]
    assert abs(got - cc.base_energy(P, X, triples=True)) <= TOL


@pytest.mark.parametrize("model", [2, 3])
def test_cc_base_expansion_matches_oracle(ws, model):
    """Orders 1-3 of the 8-site chain at U = 2 with the coupled-cluster base:
    eps - eps_base per tuple, increments, order sums and the total (which adds
    the base energy of the whole space) against the oracle's expansion."""
    P = replace_order(synth.config_hubbard(2.0, nsite=8), 3)
    res = M.Context.from_problem(P, device=0, base_model=model).run(ws)
    tri = model == 3
    ref = mbe.run(P, energy=lambda S: fci.casci_energy(P, S) - cc.base_energy(P, S, triples=tri))
    assert len(res.orders) == len(ref.orders)
    for o, ro in zip(res.orders, ref.orders):
        assert [tuple(int(x) for x in t) for t in o.tuples] == [tuple(t) for t in ro.tuples] or o.k == 0
        assert np.abs(o.eps - np.asarray(ro.eps)).max() <= 1e-10
        assert np.abs(o.dinc - np.asarray(ro.dinc)).max() <= 1e-9
    e_base = cc.base_energy(P, tuple(P.expansion_space()), triples=tri)
    assert abs(res.e_base - e_base) <= 1e-10
    assert abs(res.total - (ref.total + e_base)) <= 1e-9


def test_cc_base_full_order_is_fci(ws):
    P = synth.config_hubbard(4.0, nsite=8)
    res = M.Context.from_problem(P, device=0, base_model=3).run(ws)
    assert abs(res.total - fci.fci_energy(P)) <= 1e-9


def replace_order(P, k):
    from dataclasses import replace
    return replace(P, max_order=k)


def test_large_tuple_cooperative_launch(ws):
    """A tuple of 10 active orbitals runs on many workgroups at once (one
    cooperative launch, grid barriers between the phases): CCSD against the
    oracle in the given orbitals, CCSD(T) in the HF orbitals, and the
    expansion's full order (whose base energy of the whole space takes that
    path) equal to FCI."""
    from oracle import hf
    P = synth.small_problem(10, 2, 2, [1, 2], nvec=5, seed=7, offdiag_std=0.05)
    X = tuple(P.expansion_space())
    ctx = M.Context.from_problem(P, device=0, base_model=2)
    got = ctx.tuple_base(len(X), [X], ws)[0]
    assert abs(got - cc.base_energy(P, X)) <= TOL
    res = ctx.run(ws)
    assert abs(res.total - fci.fci_energy(P)) <= 1e-9
    _, Q, _ = hf.hf_problem(P)
    ctx3 = M.Context.from_problem(P, device=0, base_model=3)
    ctx3.hf(ws)
    got3 = ctx3.tuple_base(len(X), [X], ws)[0]
    assert abs(got3 - cc.base_energy(Q, X, triples=True)) <= 1e-8


def test_two_electrons_in_sixteen_orbitals_is_exact(ws):
    """Beyond 13 active orbitals (the cooperative launch of one tuple): for
    two electrons CCSD is exact, so the base energy of the whole 16-orbital
    space equals its CASCI energy; (T) has no triples to add, so in HF orbitals
    CCSD(T) gives FCI."""
    P = synth.small_problem(16, 1, 1, [0, 1], nvec=4, seed=3)
    X = tuple(P.expansion_space())
    ctx = M.Context.from_problem(P, device=0, base_model=2)
    assert abs(ctx.tuple_base(len(X), [X], ws)[0] - fci.casci_energy(P, X)) <= TOL
    ctx3 = M.Context.from_problem(P, device=0, base_model=3)
    ctx3.hf(ws)
    assert abs(ctx3.tuple_base(len(X), [X], ws)[0] - fci.fci_energy(P)) <= 1e-9
