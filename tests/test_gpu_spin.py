"""Spin-targeted CASCI (options.spin_shift) on the HIP path against the
oracle's total-spin module.

The library shifts every tuple's Hamiltonian by lambda S_- S_+, which
vanishes on the states of spin S = (n_alpha - n_beta) / 2 of the sector (the
lowest singlet for closed shells); the oracle picks instead, among the exact
eigenstates, the lowest one whose <S^2> is S(S+1).  On the plain 10-orbital
problem the lowest state of most tuples is a triplet (up to 0.17 E_h below
the lowest singlet), so the targeting changes the energies.  Tolerances as in
the parity tests: sigma and the diagonal within 1e-12 relative, energies
within 1e-10 E_h, increments and totals within 1e-9."""
import itertools
import json
import os

import numpy as np
import pytest

import synth
from oracle import fci, spin
from tests.test_gpu_parity import core_order_signs

torch = pytest.importorskip("torch")
import paper_1905_02786_amd as M  # noqa: E402

pytestmark = pytest.mark.gpu
GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
LAM = 1.0


@pytest.fixture(scope="module")
def ws():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return M.workspace(8 << 30)


PROBLEMS = {
    "plain": lambda: synth.config_plain(0),
    "openshell": lambda: synth.small_problem(8, 4, 2, [2, 3], nfrozen=1, nvec=6, seed=3, e_const=0.5),
}


_REF = {}


def _reference(name, S):
    """Oracle (H + lambda S_- S_+) c for seeded vectors, in the library's
    determinant signs, and the diagonal; once per case."""
    if (name, S) not in _REF:
        P = PROBLEMS[name]()
        sp = fci.cas_space(P, S)
        H = fci.hamiltonian_matrix(P, sp)
        sg = core_order_signs(sp)
        rng = np.random.default_rng(len(S) + 11)
        c = rng.standard_normal((2, sp.dim))
        ref = np.stack([sg * (H @ (sg * v) + LAM * spin.s_minus_s_plus(sp, sg * v)) for v in c])
        # the diagonal of S_- S_+: its matrix from the images of the unit vectors
        Sm = np.stack([spin.s_minus_s_plus(sp, e) for e in np.eye(sp.dim)], axis=1)
        dref = np.diag(H) + LAM * np.diag(Sm)
        _REF[(name, S)] = (P, c, ref, dref)
    return _REF[(name, S)]


@pytest.mark.parametrize("name,S", [("plain", ()), ("plain", (0, 9)), ("plain", (2, 5, 6)),
                                    ("plain", (0, 1, 5, 6)), ("openshell", (1, 5)),
                                    ("openshell", (1, 4, 5, 6))])
@pytest.mark.parametrize("variant,linked", [(1, 1), (1, 0), (1, 5), (2, 1)])
def test_spin_sigma_and_diagonal(ws, name, S, variant, linked):
    """sigma = (H + lambda S_- S_+) c and its diagonal against the oracle's H
    and S_- S_+ (every sigma form; the shift is one kernel for all)."""
    P, c, ref, dref = _reference(name, S)
    ctx = M.Context.from_problem(P, device=0, sigma_variant=variant, linked_rows=linked, spin_shift=LAM)
    sig = ctx.tuple_sigma(len(S), S, torch.tensor(c, device="cuda:0"), ws).cpu().numpy()
    scale = max(1.0, np.abs(ref).max())
    assert np.abs(sig - ref).max() <= 1e-12 * scale, np.abs(sig - ref).max()
    hd = ctx.tuple_hdiag(len(S), S, ws).cpu().numpy()
    assert np.abs(hd - dref).max() <= 1e-12 * max(1.0, np.abs(dref).max())


def test_spin_targeted_energies(ws):
    """Per-tuple energies of the plain problem's orders 0-2 with the shift:
    the oracle's lowest singlet (not its lowest state), for every tuple."""
    P = PROBLEMS["plain"]()
    ctx = M.Context.from_problem(P, device=0, spin_shift=LAM)
    X = P.expansion_space()
    moved = 0
    for k in (0, 1, 2):
        tl = list(itertools.combinations(X, k))
        e, st = ctx.solve_tuples(k, tl if k else [()], ws)
        for S, ei, si in zip(tl, e, st):
            ref = spin.casci_energy_spin(P, S)
            assert si == 0
            assert abs(ei - ref) <= 1e-10, (S, ei, ref)
            moved += abs(ref - fci.casci_energy(P, S)) > 1e-6
    assert moved > 10   # the targeting matters on this problem


def test_spin_targeted_open_shell(ws):
    """An open-shell problem (n_alpha = n_beta + 2): the shift selects the
    lowest state with S = 1 exactly (not a higher multiplet's M_s = 1
    component)."""
    P = PROBLEMS["openshell"]()
    ctx = M.Context.from_problem(P, device=0, spin_shift=LAM)
    for S in [(), (1,), (5,), (1, 5), (4, 6)]:
        e, st = ctx.solve_tuples(len(S), [S] if S else [()], ws)
        ref = spin.casci_energy_spin(P, S)
        assert st[0] == 0 and abs(e[0] - ref) <= 1e-10, (S, e[0], ref)


def test_spin_targeted_mbe_matches_oracle(ws):
    """The full-order MBE of the plain problem with spin-targeted energies:
    every tuple, increment and order sum against the oracle's
    (tests/golden/plain_spin.json, written from the oracle alone)."""
    path = os.path.join(GOLDEN, "plain_spin.json")
    if not os.path.exists(path):
        pytest.skip("plain_spin.json not generated")
    with open(path) as f:
        g = json.load(f)
    P = PROBLEMS["plain"]()
    res = M.Context.from_problem(P, device=0, spin_shift=LAM).run(ws)
    assert len(res.orders) == len(g["orders"])
    for o, go in zip(res.orders, g["orders"]):
        assert [tuple(t) for t in o.tuples] == [tuple(t) for t in go["tuples"]]
        assert np.abs(np.asarray(o.eps) - np.asarray(go["eps"])).max() <= 1e-10
        assert np.abs(np.asarray(o.dinc) - np.asarray(go["dinc"])).max() <= 1e-9
        assert abs(o.order_sum - go["order_sum"]) <= 1e-9
    assert abs(res.total - g["total"]) <= 1e-9


def test_spin_shift_off_is_unchanged(ws):
    """spin_shift = 0 (the default) reproduces the plain lowest eigenvalues."""
    P = PROBLEMS["plain"]()
    tl = [(0,), (5,), (0, 9)]
    for S in tl:
        e, _ = M.Context.from_problem(P, device=0).solve_tuples(len(S), [S], ws)
        assert abs(e[0] - fci.casci_energy(P, S)) <= 1e-10
