"""Parity of the HIP RDM adjoint (through the C ABI and the autograd wrapper)
with the CPU oracle's density matrices and MBE gradients.

Tolerance: gradients and density matrices within 1e-7 (max abs); the
Davidson runs with a tight residual (1e-9) so that its vectors carry no error
at that level."""
import os

import numpy as np
import pytest

import synth
from oracle import fci, mbe as ombe, rdm as ordm

torch = pytest.importorskip("torch")
import paper_1905_02786_amd as M  # noqa: E402
from paper_1905_02786_amd.autograd import MBEFCIEnergy  # noqa: E402

pytestmark = pytest.mark.gpu
GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
TIGHT = dict(r_tol=1e-9, e_tol=1e-12, max_iter=400)


@pytest.fixture(scope="module")
def ws():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return M.workspace(8 << 30)


RDM_CASES = [
    ("plain", ()), ("plain", (0,)), ("plain", (2, 5, 6)), ("plain", (0, 1, 5, 6)),
    ("sweep", (1, 9)), ("sweep", (2, 10, 13)),
    ("openshell", ()), ("openshell", (1, 5)),
]
PROBLEMS = {
    "plain": lambda: synth.config_plain(0),
    "sweep": lambda: synth.config_sweep(0),
    "openshell": lambda: synth.small_problem(8, 4, 2, [2, 3], nfrozen=1, nvec=6, seed=3, e_const=0.5),
}


@pytest.mark.parametrize("name,S", RDM_CASES)
def test_tuple_rdm_matches_oracle(ws, name, S):
    P = PROBLEMS[name]()
    ctx = M.Context.from_problem(P, device=0, **TIGHT)
    e, g1, g2 = ctx.tuple_rdm(len(S), S, ws)
    e_ref, v, sp = fci.casci_energy(P, S, want_vector=True)
    r1, r2 = ordm.rdm12(P, sp, v)
    print(f"{name} {S} dim {sp.dim}: |dgamma| {np.abs(g1 - r1).max():.1e} |dGamma| {np.abs(g2 - r2).max():.1e}")
    assert abs(e - e_ref) <= 1e-10
    assert np.abs(g1 - r1).max() <= 1e-7
    assert np.abs(g2 - r2).max() <= 1e-7
    # the energy rebuilt from the device density matrices
    assert abs(ordm.energy_from_rdms(P, g1, g2) - e) <= 1e-9


def _golden():
    path = os.path.join(GOLDEN, "gradients.npz")
    if not os.path.exists(path):
        pytest.skip("gradients.npz not generated")
    return np.load(path)


@pytest.mark.parametrize("name,K", [("plain", 2), ("plain", 4), ("plain", 0),
                                    ("hubbard4", 2), ("hubbard4", 4), ("hubbard4", 0)])
def test_mbe_gradient_matches_oracle(ws, name, K):
    g = _golden()
    P = synth.config_plain(0) if name == "plain" else synth.config_hubbard(4.0)
    ctx = M.Context.from_problem(P, device=0, max_order=K, **TIGHT)
    res, handle = ctx.run(ws, keep=True)
    key = f"{name}_K{K if K else 'full'}"
    assert abs(res.total - float(g[key + "_E"][0])) <= 1e-9
    gh, ge = ctx.backward(handle, ws)
    dh, de = np.abs(gh - g[key + "_h"]).max(), np.abs(ge - g[key + "_eri"]).max()
    print(f"{key}: |dE/dh - oracle| {dh:.1e}  |dE/d(pq|rs) - oracle| {de:.1e}")
    assert dh <= 1e-7 and de <= 1e-7


def test_full_order_gradient_is_fci_rdm(ws):
    P = synth.small_problem(8, 3, 3, [2, 3], nfrozen=1, nvec=6, seed=11)
    ctx = M.Context.from_problem(P, device=0, **TIGHT)
    res, handle = ctx.run(ws, keep=True)
    gh, ge = ctx.backward(handle, ws)
    e, v, sp = fci.casci_energy(P, tuple(P.expansion_space()), want_vector=True)
    r1, r2 = ordm.rdm12(P, sp, v)
    assert abs(res.total - e) <= 1e-9
    assert np.abs(gh - r1).max() <= 1e-7
    assert np.abs(ge - 0.5 * r2).max() <= 1e-7


def test_autograd_and_finite_differences(ws):
    """torch.autograd through MBEFCIEnergy equals the library backward, and a
    central difference of the device energy along symmetry orbits (tuple set
    fixed by a = 0, max order 2) matches it."""
    P = synth.small_problem(7, 3, 3, [2, 3], nfrozen=1, nvec=5, seed=4)
    spec = dict(nalpha=P.nalpha, nbeta=P.nbeta, nfrozen=P.nfrozen, ref=P.ref, a=0.0, max_order=2)
    h = torch.tensor(P.h, dtype=torch.float64, requires_grad=True)
    eri = torch.tensor(P.eri, dtype=torch.float64, requires_grad=True)
    E = MBEFCIEnergy.apply(h, eri, spec, ws)
    E.backward()
    ctx = M.Context.from_problem(P, device=0, a=0.0, max_order=2)
    res, handle = ctx.run(ws, keep=True)
    gh, ge = ctx.backward(handle, ws)
    # the same tuples, solved again with the same (tightened) options: equal up
    # to the order of the device's atomic adds
    assert np.abs(h.grad.numpy() - gh).max() <= 1e-12
    assert np.abs(eri.grad.numpy() - ge).max() <= 1e-12
    # against the oracle's gradient of the same truncated expansion
    from oracle import rdm as ordm2
    ref = ombe.run(P, max_order=2)
    rh, re_ = ordm2.mbe_gradient(P, ref)
    assert np.abs(gh - rh).max() <= 1e-7 and np.abs(ge - re_).max() <= 1e-7

    def energy(hh, ee):
        c = M.Context(device=0)
        c.set_hamiltonian(hh, ee)
        c.set_spaces(P.nalpha, P.nbeta, P.nfrozen, P.ref)
        c.set_options(a=0.0, max_order=2, **TIGHT)
        return c.run(ws).total

    step = 1e-4
    for (p, q) in [(1, 4), (3, 3)]:
        hp, hm = P.h.copy(), P.h.copy()
        for a_, b_ in {(p, q), (q, p)}:
            hp[a_, b_] += step
            hm[a_, b_] -= step
        fd = (energy(hp, P.eri) - energy(hm, P.eri)) / (2 * step)
        an = gh[p, q] + (gh[q, p] if p != q else 0.0)
        assert abs(fd - an) <= 1e-6, (p, q, fd, an)
    p, q, r, s = 1, 2, 4, 5
    orbit = {(p, q, r, s), (q, p, r, s), (p, q, s, r), (q, p, s, r),
             (r, s, p, q), (s, r, p, q), (r, s, q, p), (s, r, q, p)}
    ep, em = P.eri.copy(), P.eri.copy()
    for o in orbit:
        ep[o] += step
        em[o] -= step
    fd = (energy(P.h, ep) - energy(P.h, em)) / (2 * step)
    an = sum(ge[o] for o in orbit)
    assert abs(fd - an) <= 1e-6, (fd, an)


def _pack8(eri):
    """(pq|rs) as its unique elements: P = p(p+1)/2 + q (p >= q), element
    [P(P+1)/2 + R] for P >= R."""
    n = eri.shape[0]
    pairs = [(p, q) for p in range(n) for q in range(p + 1)]
    out = np.zeros(len(pairs) * (len(pairs) + 1) // 2)
    for P, (p, q) in enumerate(pairs):
        for R in range(P + 1):
            r, s = pairs[R]
            out[P * (P + 1) // 2 + R] = eri[p, q, r, s]
    return out


def _orbit_sums(ge):
    """Packed-layout gradient from a full-layout one: per packed element the
    sum over the distinct quadruples of its orbit."""
    n = ge.shape[0]
    idx = {}
    for p in range(n):
        for q in range(p + 1):
            idx[(p, q)] = idx[(q, p)] = p * (p + 1) // 2 + q
    npair = n * (n + 1) // 2
    out = np.zeros(npair * (npair + 1) // 2)
    for p, q, r, s in np.ndindex(n, n, n, n):
        P, R = idx[(p, q)], idx[(r, s)]
        if P < R:
            P, R = R, P
        out[P * (P + 1) // 2 + R] += ge[p, q, r, s]
    return out


@pytest.mark.parametrize("name,K", [("plain", 2), ("plain", 0), ("hubbard4", 4)])
def test_forward_gradient_default_options(ws, name, K):
    """Default Davidson options: the forward run with options.gradient = 1
    forms the gradient itself (the last order on the device with weight 1, the
    lower orders weighted after the lists are known), backward() re-solves
    nothing, and the re-solving backward of a plain run agrees; both within
    1e-7 of the oracle."""
    g = _golden()
    P = synth.config_plain(0) if name == "plain" else synth.config_hubbard(4.0)
    key = f"{name}_K{K if K else 'full'}"
    ctx = M.Context.from_problem(P, device=0, max_order=K, gradient=1)
    res, handle = ctx.run(ws, keep=True)
    assert abs(res.total - float(g[key + "_E"][0])) <= 1e-9
    gh, ge = ctx.backward(handle, ws)
    dh, de = np.abs(gh - g[key + "_h"]).max(), np.abs(ge - g[key + "_eri"]).max()
    ctx2 = M.Context.from_problem(P, device=0, max_order=K)
    res2, handle2 = ctx2.run(ws, keep=True)
    gh2, ge2 = ctx2.backward(handle2, ws)
    dh2, de2 = np.abs(gh2 - g[key + "_h"]).max(), np.abs(ge2 - g[key + "_eri"]).max()
    print(f"{key}: forward-gradient |dh| {dh:.1e} |deri| {de:.1e}; re-solving backward |dh| {dh2:.1e} |deri| {de2:.1e}")
    assert dh <= 1e-7 and de <= 1e-7
    assert dh2 <= 1e-7 and de2 <= 1e-7


def test_packed_layout_gradient(ws):
    """Integrals given in the packed 8-fold layout: dE/d(pq|rs) comes back in
    that layout, each element the derivative with respect to the one stored
    number (the orbit sum of the full-layout gradient)."""
    g = _golden()
    P = synth.config_plain(0)
    ctx = M.Context(device=0)
    ctx.set_hamiltonian(P.h, _pack8(P.eri))
    ctx.set_spaces(P.nalpha, P.nbeta, P.nfrozen, P.ref)
    ctx.set_options(a=0.0, max_order=2)
    res, handle = ctx.run(ws, keep=True)
    assert abs(res.total - float(g["plain_K2_E"][0])) <= 1e-9
    gh, gp = ctx.backward(handle, ws, gE=2.0)
    assert gp.shape == (55 * 56 // 2,)
    ref = 2.0 * _orbit_sums(g["plain_K2_eri"])
    print(f"packed: |dh| {np.abs(gh - 2.0 * g['plain_K2_h']).max():.1e} |dpacked| {np.abs(gp - ref).max():.1e}")
    assert np.abs(gh - 2.0 * g["plain_K2_h"]).max() <= 2e-7
    assert np.abs(gp - ref).max() <= 1e-6
