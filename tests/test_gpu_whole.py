"""Whole-tuple mode (options.whole_dim): one workgroup runs the complete
Davidson solve of a small tuple in one launch.  Energies against the oracle's
CASCI energies (Sec. 2), at the bar of the other parity tests: 1e-10 E_h per
tuple; the batched path (whole_dim = 0) gives the same energies within that
bar, and a run in whole-tuple mode repeats bitwise."""
import itertools

import numpy as np
import pytest

import synth
from oracle import fci, spin

torch = pytest.importorskip("torch")
import paper_1905_02786_amd as M  # noqa: E402

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ws():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return M.workspace(8 << 30)


def _tuples(P, k, lo, hi):
    out = []
    for S in itertools.combinations(P.expansion_space(), k):
        d = fci.cas_space(P, S).dim
        if lo <= d <= hi:
            out.append(S)
    return out


def _whole_classes(ctx):
    return [c for c in ctx.class_stats() if c["kernel"] == 6]


@pytest.mark.parametrize("name,k", [("plain", 3), ("plain", 5), ("plain", 6), ("hubbard8", 4), ("hubbard8", 6),
                                    ("sweep", 1)])
def test_whole_mode_matches_oracle(ws, name, k):
    """Every tuple of the order with at most 4900 determinants (the mode's
    largest setting, whole_dim = 4900; (8e,8o) of the plain problem is
    exactly 4900), against the oracle; and against the batched path."""
    P = {"plain": lambda: synth.config_plain(0), "hubbard8": lambda: synth.config_hubbard(8.0),
         "sweep": lambda: synth.config_sweep(0)}[name]()
    tl = _tuples(P, k, 1, 4900)
    assert tl
    ctx = M.Context.from_problem(P, device=0, whole_dim=4900)
    e, st = ctx.solve_tuples(k, tl, ws)
    assert (st == 0).all()
    assert ctx.stats()["whole_batches"] > 0 and _whole_classes(ctx)
    assert all(c["kernel"] == 6 for c in ctx.class_stats())
    ref = np.array([fci.casci_energy(P, S) for S in tl])
    print(f"{name} order {k}: {len(tl)} tuples, dims up to "
          f"{max(fci.cas_space(P, S).dim for S in tl)}, max |dE| {np.abs(e - ref).max():.2e}", flush=True)
    assert np.abs(e - ref).max() <= 1e-10
    e0, st0 = M.Context.from_problem(P, device=0, whole_dim=0).solve_tuples(k, tl, ws)
    assert (st0 == 0).all() and np.abs(e - e0).max() <= 1e-10
    e2, _ = ctx.solve_tuples(k, tl, ws)
    assert np.array_equal(e, e2)


@pytest.mark.parametrize("opts", [dict(max_space=3), dict(max_space=4, restart_keep=1),
                                  dict(max_space=5, restart_keep=2), dict(max_space=32, pspace=0),
                                  dict(pspace=0), dict(pspace=7), dict(batched=0)])
def test_whole_mode_settings(ws, opts):
    """Restarts (small subspaces, with and without the previous Ritz
    vector), the 32-vector form of the second pass, the diagonal
    preconditioner alone, a small P space, and one tuple per launch."""
    P = synth.config_hubbard(8.0)
    tl = _tuples(P, 5, 400, 4900)[::3]
    ctx = M.Context.from_problem(P, device=0, max_iter=1000, whole_dim=4900, **opts)
    e, st = ctx.solve_tuples(5, tl, ws)
    assert (st == 0).all()
    assert ctx.stats()["whole_batches"] > 0
    ref = np.array([fci.casci_energy(P, S) for S in tl])
    assert np.abs(e - ref).max() <= 1e-10


def test_whole_mode_spin_shift(ws):
    """The spin level shift inside the whole-tuple sigma: the lowest
    singlets of the plain problem's order-3 tuples."""
    P = synth.config_plain(0)
    tl = _tuples(P, 3, 1, 4900)
    ctx = M.Context.from_problem(P, device=0, spin_shift=1.0, whole_dim=4900)
    e, st = ctx.solve_tuples(3, tl, ws)
    assert (st == 0).all() and ctx.stats()["whole_batches"] > 0
    ref = np.array([spin.casci_energy_spin(P, S) for S in tl])
    assert np.abs(e - ref).max() <= 1e-10


def test_whole_mode_full_expansion(ws):
    """The plain problem's whole expansion with the default settings (classes
    up to 1225 determinants in whole-tuple mode, the rest batched) equals FCI
    and the batched path's total."""
    P = synth.config_plain(0)
    ctx = M.Context.from_problem(P, device=0)
    res = ctx.run(ws)
    assert ctx.stats()["whole_batches"] > 0
    r0 = M.Context.from_problem(P, device=0, whole_dim=0).run(ws)
    e_fci = fci.casci_energy(P, tuple(P.expansion_space()))
    assert abs(res.total - e_fci) <= 1e-9 and abs(res.total - r0.total) <= 1e-9
