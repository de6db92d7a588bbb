"""Base-model expansion (options.base_model = 1; MBE-FCI-b of Sec. 4.2.1 with
a second-order base in place of CCSD(T)) against the oracle: per-tuple base
energies (oracle/base.py, brute force over the CAS determinants; the library
sums over excitations) within 1e-11, the expansion of eps - eps_base and its
total within the parity tests' 1e-10 / 1e-9, full order equal to FCI."""
import itertools
import json
import os

import numpy as np
import pytest

import synth
from oracle import base, fci, mbe

torch = pytest.importorskip("torch")
import paper_1905_02786_amd as M  # noqa: E402

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ws():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return M.workspace(2 << 30)


PROBLEMS = {
    "hubbard2": lambda: synth.config_hubbard(2.0),
    "hubbard4": lambda: synth.config_hubbard(4.0),
    "open8": lambda: synth.small_problem(8, 4, 2, [2, 3], nfrozen=1, nvec=6, seed=3, e_const=0.5),
}


@pytest.mark.parametrize("name", list(PROBLEMS))
def test_tuple_base_energies_match_oracle(ws, name):
    P = PROBLEMS[name]()
    ctx = M.Context.from_problem(P, device=0)
    X = P.expansion_space()
    worst = 0.0
    for k in (0, 1, 2, 3):
        tl = list(itertools.combinations(X, k)) if k else [()]
        got = ctx.tuple_base(k, tl, ws)
        ref = np.array([base.base_energy(P, S) for S in tl])
        worst = max(worst, float(np.abs(got - ref).max()))
    full = ctx.tuple_base(len(X), [tuple(X)], ws)[0]
    worst = max(worst, abs(full - base.base_energy(P, tuple(X))))
    print(f"{name}: max |d eps_base| {worst:.1e}", flush=True)
    assert worst <= 1e-11


def test_intruder_is_reported(ws):
    """The plain problem's orbitals are not ordered like canonical ones: an
    excitation lowers the zeroth-order energy, and the library refuses."""
    P = synth.config_plain(0)
    with pytest.raises(ValueError, match="base model"):
        base.base_energy(P, ())
    ctx = M.Context.from_problem(P, device=0)
    with pytest.raises(M.MBEFCIError, match="intruder"):
        ctx.tuple_base(0, [()], ws)
    with pytest.raises(M.MBEFCIError):
        M.Context.from_problem(P, device=0, base_model=1).run(ws)


@pytest.mark.parametrize("nsite,U", [(8, 2.0), (10, 4.0)])
def test_base_model_expansion_matches_oracle(ws, nsite, U):
    P = synth.config_hubbard(U, nsite=nsite)
    res = M.Context.from_problem(P, device=0, base_model=1).run(ws)
    # CASCI energies: the oracle's (for 10 sites from its stored full-order run)
    golden = {}
    if nsite == 10:
        with open(os.path.join(os.path.dirname(__file__), "golden", f"hubbard_U{U:g}.json")) as f:
            for o in json.load(f)["unscreened"]["orders"]:
                for t, e in zip(o["tuples"], o["eps"]):
                    golden[tuple(t)] = e

    def eps(S):
        e = golden[tuple(S)] if golden else fci.casci_energy(P, S)
        return e - base.base_energy(P, S)
    ref = mbe.run(P, energy=eps)
    e_base = base.base_energy(P, tuple(P.expansion_space()))
    assert abs(res.e_base - e_base) <= 1e-11
    assert len(res.orders) == len(ref.orders)
    for o, ro in zip(res.orders, ref.orders):
        assert [tuple(int(x) for x in t) for t in o.tuples] == [tuple(t) for t in ro.tuples] or o.k == 0
        assert np.abs(o.eps - np.asarray(ro.eps)).max() <= 1e-10
        assert np.abs(o.dinc - np.asarray(ro.dinc)).max() <= 1e-9
    assert abs(res.total - (ref.total + e_base)) <= 1e-9
    e_fci = golden[tuple(P.expansion_space())] if golden else fci.fci_energy(P)
    assert abs(res.total - e_fci) <= 1e-9     # full order: the base energies cancel


def test_base_model_screened_expansion_matches_oracle(ws):
    """With screening that removes tuples (a = 5 on the weakly coupled
    problem) the screened increments are those of eps - eps_base: the tuple
    lists equal the oracle's (every |dinc| lies at least 6 % from its
    threshold), the energies agree to the parity bounds."""
    P = synth.config_weak()
    res = M.Context.from_problem(P, device=0, base_model=1).run(ws)
    ref = mbe.run(P, energy=lambda S: fci.casci_energy(P, S) - base.base_energy(P, S))
    assert len(res.orders) == len(ref.orders)
    for o, ro in zip(res.orders, ref.orders):
        assert [tuple(int(x) for x in t) for t in o.tuples] == [tuple(t) for t in ro.tuples] or o.k == 0
        assert np.abs(o.eps - np.asarray(ro.eps)).max() <= 1e-10
        assert np.abs(o.dinc - np.asarray(ro.dinc)).max() <= 1e-9
    e_base = base.base_energy(P, base.full_space_tuple(P))
    assert abs(res.e_base - e_base) <= 1e-11
    assert abs(res.total - (ref.total + e_base)) <= 1e-9


def test_base_model_streamed_last_order(ws):
    """The streamed last order subtracts the base energies too and the
    closed result equals the one-call run."""
    P = synth.config_hubbard(2.0, nsite=8)
    one = M.Context.from_problem(P, device=0, base_model=1).run(ws)
    ctx = M.Context.from_problem(P, device=0, base_model=1, stream_last=1)
    part, h = ctx.run(ws, keep=True)
    nt = len(part.orders[-1].tuples)
    for first in range(3):
        ctx.order_solve(h, first, 3, len(range(first, nt, 3)), ws)
    res = ctx.order_close(h)
    assert abs(res.total - one.total) <= 1e-12
    assert abs(res.e_base - one.e_base) == 0.0
    assert np.abs(res.orders[-1].eps - one.orders[-1].eps).max() <= 1e-12


def test_gradient_with_base_model_is_refused(ws):
    P = synth.config_hubbard(2.0, nsite=8)
    with pytest.raises(M.MBEFCIError):
        M.Context.from_problem(P, device=0, base_model=1, gradient=1).run(ws)
