"""The allocation-free entry point mbefci_solve_tuples_noalloc (static device
workspace) against mbefci_solve_tuples with a caller's workspace: the same
energies (per-tuple Davidson does not depend on the batch) within 1e-10 E_h
on two calls in a row, the second with a smaller input, and ENOMEM for a
tuple larger than the static workspace."""
import itertools

import numpy as np
import pytest

import synth

torch = pytest.importorskip("torch")
import paper_1905_02786_amd as M  # noqa: E402

pytestmark = pytest.mark.gpu


def test_noalloc_matches_workspace_entry_point():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    P = synth.config_plain(0)
    X = P.expansion_space()
    ws = M.workspace(2 << 30)
    ctx = M.Context.from_problem(P, device=0)
    for k in (4, 2):     # 70 tuples, then 28 smaller ones
        tl = list(itertools.combinations(X, k))
        print(f"order {k}: {len(tl)} tuples", flush=True)
        e0, s0 = ctx.solve_tuples(k, tl, ws)
        e1, s1 = ctx.solve_tuples_noalloc(k, tl)
        assert (s0 == 0).all() and (s1 == 0).all()
        assert np.abs(e1 - e0).max() <= 1e-10, np.abs(e1 - e0).max()
    # a tuple of 853776 determinants needs more than the 128 MiB
    L = synth.config_large(0)
    ctxl = M.Context.from_problem(L, device=0)
    with pytest.raises(M.MBEFCIError) as ex:
        ctxl.solve_tuples_noalloc(4, [(0, 1, 10, 11)])
    assert ex.value.code == -2
