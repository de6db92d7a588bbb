"""CASSCF expansion reference (mbefci_casscf) against the oracle's CASSCF
orbitals and the expansion in them (tests/golden/casscf.json, written from
oracle/casscf.py and oracle/mbe.py alone).

Tolerances: the CASSCF energy is stationary in the orbitals, so it agrees to
1e-9; the orbitals are converged to a gradient of 1e-10 on both sides, i.e.
to about 1e-10 / 0.05 = 2e-9 in the rotation angles (0.05 is the smallest
diagonal Hessian estimate used), and the tuples' energies, which are not
stationary in the orbitals, follow that to a few 1e-9 (bound 1e-8).  Orbitals
are compared up to the sign of each (the sign rule picks the largest entry,
which two nearly equal entries could flip), the active ones as a space."""
import json
import os

import numpy as np
import pytest

import synth
from oracle import fci

torch = pytest.importorskip("torch")
import paper_1905_02786_amd as M  # noqa: E402

pytestmark = pytest.mark.gpu
GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "casscf.json")

PROBLEMS = {
    "plain": lambda: synth.config_plain(0),
    "small7": lambda: synth.small_problem(7, 3, 3, [2, 3], nfrozen=1, nvec=6, seed=11, vec_std=0.15,
                                          offdiag_std=0.2),
    "open8": lambda: synth.small_problem(8, 4, 2, [2, 3], nfrozen=1, nvec=6, seed=3, e_const=0.5),
    "plain_singlet": lambda: synth.config_plain(0),
}
# the singlet-targeted case: the reference state and every tuple's state are
# the lowest singlets (options.spin_shift, the oracle's spin module)
SPIN_SHIFT = {"plain_singlet": 1.0}


@pytest.fixture(scope="module")
def ws():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return M.workspace(4 << 30)


@pytest.fixture(scope="module")
def golden():
    if not os.path.exists(GOLDEN):
        pytest.skip("casscf.json not generated")
    with open(GOLDEN) as f:
        return json.load(f)


@pytest.mark.parametrize("key", ["small7", "open8", "plain", "plain_singlet"])
def test_casscf_orbitals_and_expansion_match_oracle(ws, golden, key):
    if key not in golden:
        pytest.skip(f"{key} not in casscf.json")
    g = golden[key]
    P = PROBLEMS[key]()
    ctx = M.Context.from_problem(P, device=0, spin_shift=SPIN_SHIFT.get(key, 0.0))
    out = ctx.casscf(ws, g_tol=1e-10)
    print(f"{key}: CASSCF {out['energy']:.12f} (oracle {g['e_casscf']:.12f}, start {g['e_casci_start']:.6f}), "
          f"{out['iterations']} steps", flush=True)
    assert abs(out["energy"] - g["e_casscf"]) <= 1e-9
    U, Ug = out["U"], np.array(g["U"])
    assert np.abs(U.T @ U - np.eye(P.norb)).max() <= 1e-12
    # core and virtual orbitals one by one; the active orbitals as a space
    # (their natural occupations can be degenerate -- [1, 1] for the plain
    # problem's open-shell reference state -- and no tuple energy depends on
    # rotations inside [Pi], which every CAS contains)
    act = sorted(P.ref)
    cv = [p for p in range(P.norb) if p not in act]
    sg = np.sign(np.sum(U * Ug, axis=0))
    assert np.abs((U * sg - Ug)[:, cv]).max() <= 1e-6
    PA, PAg = U[:, act] @ U[:, act].T, Ug[:, act] @ Ug[:, act].T
    assert np.abs(PA - PAg).max() <= 1e-6
    h, eri, c = ctx.hamiltonian()
    D = np.diag(sg)
    assert np.abs((D @ h @ D - np.array(g["h"]))[np.ix_(cv, cv)]).max() <= 1e-7
    assert c == P.e_const
    # the expansion in the CASSCF orbitals
    res = ctx.run(ws)
    assert len(res.orders) == len(g["orders"])
    worst = 0.0
    for o, go in zip(res.orders, g["orders"]):
        assert [list(map(int, t)) for t in o.tuples] == [list(t) for t in go["tuples"]] or o.k == 0
        assert (o.status == 0).all()
        worst = max(worst, float(np.abs(o.eps - np.array(go["eps"])).max()))
        assert np.abs(o.dinc - np.array(go["dinc"])).max() <= 1e-8
    print(f"{key}: max |d eps| {worst:.1e}, total {res.total:.12f} (oracle {g['total']:.12f})")
    assert worst <= 1e-8
    assert abs(res.total - g["total"]) <= 1e-8
    if g.get("fci") is not None:
        assert abs(res.total - g["fci"]) <= 1e-8   # full order: FCI in any orbitals


def test_casscf_from_canonical_orbitals_stays(ws):
    """A second call starts at the optimum: no rotation beyond signs, the
    same energy."""
    P = PROBLEMS["small7"]()
    ctx = M.Context.from_problem(P, device=0)
    e1 = ctx.casscf(ws, g_tol=1e-10)["energy"]
    out = ctx.casscf(ws, g_tol=1e-10)
    assert abs(out["energy"] - e1) <= 1e-10
    assert np.abs(np.abs(out["U"]) - np.eye(P.norb)).max() <= 1e-6


def test_casscf_energy_is_the_reference_casci_in_its_orbitals(ws):
    """The energy returned equals the reference-space CASCI of the rotated
    Hamiltonian (order 0 of a later expansion) and lies below the starting
    CASCI."""
    P = PROBLEMS["small7"]()
    ctx = M.Context.from_problem(P, device=0)
    out = ctx.casscf(ws, g_tol=1e-10)
    e0, st = ctx.solve_tuples(0, [()], ws)
    assert st[0] == 0 and abs(e0[0] - out["energy"]) <= 1e-10
    assert out["energy"] < fci.casci_energy(P, ()) - 1e-4
