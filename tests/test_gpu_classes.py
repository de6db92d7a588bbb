"""Parity at the large shape classes of the order sweep and of the
60-orbital problem (n_A = 10 ... 12, dims up to 853776): CASCI energies within
1e-10 E_h and density matrices within 1e-7 of stored oracle values
(tests/golden/class_samples.json, rdm_large.npz; written by make_golden.py,
which calls only the oracle).  The stored gap to the second root backs the
residual tolerance: the Ritz value error is about |r|^2 / gap."""
import json
import os
from collections import defaultdict

import numpy as np
import pytest

import synth

torch = pytest.importorskip("torch")
import paper_1905_02786_amd as M  # noqa: E402

pytestmark = pytest.mark.gpu
GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
TIGHT = dict(r_tol=1e-9, e_tol=1e-12, max_iter=600)

PROBLEMS = {"sweep": lambda: synth.config_sweep(0), "sweep01": lambda: synth.config_sweep(0, vec_std=0.1),
            "large": lambda: synth.config_large(0)}


@pytest.fixture(scope="module")
def ws():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return M.workspace(32 << 30)


def _load(name):
    path = os.path.join(GOLDEN, name)
    if not os.path.exists(path):
        pytest.skip(f"{name} not generated")
    return path


@pytest.mark.parametrize("problem", ["sweep", "sweep01", "large"])
def test_class_sample_energies(ws, problem):
    with open(_load("class_samples.json")) as f:
        samples = [s for s in json.load(f)["samples"] if s["problem"] == problem]
    if not samples:
        pytest.skip("no samples")
    P = PROBLEMS[problem]()
    ctx = M.Context.from_problem(P, device=0)
    by_order = defaultdict(list)
    for s in samples:
        by_order[len(s["tuple"])].append(s)
    for k, lst in sorted(by_order.items()):
        tl = [tuple(s["tuple"]) for s in lst]
        print(f"{problem} order {k}: {len(tl)} tuples, dims {[s['dim'] for s in lst]}", flush=True)
        e, st = ctx.solve_tuples(k, tl if k else [()], ws)
        for s, ei, si in zip(lst, e, st):
            gap = (s["eps1"] - s["eps"]) if s.get("eps1") is not None else float("nan")
            print(f"  {tuple(s['tuple'])} ({s['na']}a{s['nb']}b, {s['n_active']}o) dE = {ei - s['eps']:+.1e}, "
                  f"gap {gap:.3e}", flush=True)
            assert si == 0
            assert abs(ei - s["eps"]) <= 1e-10, (s["tuple"], ei, s["eps"])


def test_rdm_large_classes(ws):
    g = np.load(_load("rdm_large.npz"))
    tags = sorted({k.rsplit("_", 1)[0] for k in g.files if k.endswith("_eps")})
    for tag in tags:
        problem, rest = tag.split("_", 1)
        S = tuple(int(x) for x in rest.split("_"))
        P = PROBLEMS[problem]()
        ctx = M.Context.from_problem(P, device=0, **TIGHT)
        e, g1, g2 = ctx.tuple_rdm(len(S), S, ws)
        A = g[tag + "_active"]
        d1 = np.abs(g1[np.ix_(A, A)] - g[tag + "_gamma"]).max()
        d2 = np.abs(g2[np.ix_(A, A, A, A)] - g[tag + "_Gamma"]).max()
        eps = g[tag + "_eps"]
        print(f"{tag}: n_A {len(A)}, dE {e - eps[0]:+.1e}, gap {eps[1] - eps[0]:.3e}, |dgamma| {d1:.1e}, "
              f"|dGamma| {d2:.1e}", flush=True)
        assert abs(e - eps[0]) <= 1e-10
        assert d1 <= 1e-7 and d2 <= 1e-7
