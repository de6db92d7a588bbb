"""Write the stored expected values used by the GPU parity tests.

Every value here comes from the CPU oracle (``oracle/``) run on the seeded
synthetic inputs of ``synth``; nothing is read from the HIP path.

    python tests/golden/make_golden.py [name ...]

Outputs (JSON, one file per workload) next to this script:
  plain_s0.json        full-order MBE of the plain 10-orbital problem + FCI
  hubbard_U{2,4,8}.json  full-order MBE of the 10-site chain, a = 0 and a = 5.0
  sweep_sample.json    sampled CASCI energies of the 24-orbital order sweep
  large_sample.json    sampled CASCI energies of the 60-orbital problem
  gradients.npz        MBE gradients (h, (pq|rs)) at orders 2, 4 and full
"""
from __future__ import annotations

import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import synth  # noqa: E402
from oracle import fci, mbe  # noqa: E402

HERE = os.path.dirname(os.path.abspath(__file__))


def mbe_json(P, res, extra=None):
    d = {"name": P.name, "a": P.a, "orders": []}
    for o in res.orders:
        d["orders"].append({"k": o.k, "tuples": [list(t) for t in o.tuples], "eps": o.eps,
                            "dinc": o.dinc, "order_sum": o.order_sum})
    d["total"] = res.total
    if extra:
        d.update(extra)
    return d


def write(name, d):
    with open(os.path.join(HERE, name), "w") as f:
        json.dump(d, f, indent=0)
    print("wrote", name, flush=True)


def plain():
    P = synth.config_plain(0)
    t = time.time()
    cache = {}

    def energy(S):
        if S not in cache:
            cache[S] = fci.casci_energy(P, S)
        return cache[S]
    res = mbe.run(P, energy=energy)
    e_fci = cache[tuple(P.expansion_space())]
    write("plain_s0.json", mbe_json(P, res, {"fci": e_fci, "seconds": time.time() - t}))


def hubbard():
    for U in (2.0, 4.0, 8.0):
        t = time.time()
        P = synth.config_hubbard(U=U)
        cache = {}

        def energy(S):
            if S not in cache:
                cache[S] = fci.casci_energy(P, S)
            return cache[S]
        res0 = mbe.run(P, energy=energy)
        P5 = synth.config_hubbard(U=U, a=5.0)
        res5 = mbe.run(P5, energy=energy)
        d = {"U": U, "unscreened": mbe_json(P, res0), "screened": mbe_json(P5, res5),
             "fci": cache[tuple(P.expansion_space())], "seconds": time.time() - t}
        write(f"hubbard_U{U:g}.json", d)


def sample(P, picks, fname):
    """picks: list of tuples; stores eps for each (oracle CASCI)."""
    out = []
    for S in picks:
        t = time.time()
        sp = fci.cas_space(P, S)
        e = fci.casci_energy(P, S)
        out.append({"tuple": list(S), "eps": e, "dim": sp.dim, "seconds": time.time() - t})
        print(fname, S, sp.dim, e, f"{time.time() - t:.1f}s", flush=True)
    write(fname, {"name": P.name, "samples": out})


def sweep():
    P = synth.config_sweep(0)
    X = P.expansion_space()
    rng = np.random.default_rng(1)
    picks = [()]
    for k in range(1, 6):
        import itertools
        allt = list(itertools.combinations(X, k))
        byclass = {}
        for S in allt:
            sp = fci.cas_space(P, S)
            byclass.setdefault((sp.na, sp.nb, len(sp.active)), []).append((S, sp.dim))
        for key in sorted(byclass):
            cand = byclass[key]
            if cand[0][1] > 30000:
                continue
            n = 2 if k >= 4 else 3
            for i in rng.choice(len(cand), size=min(n, len(cand)), replace=False):
                picks.append(tuple(int(x) for x in cand[int(i)][0]))
    sample(P, picks, "sweep_sample.json")


def large():
    P = synth.config_large(0)
    X = P.expansion_space()
    picks = [(), (X[0],), (X[5],), (X[1], X[7])]
    sample(P, picks, "large_sample.json")


def gradients():
    """Oracle MBE gradients (h and full (pq|rs)) of the plain problem and the
    U/t = 4 chain at truncation orders 2, 4 and full order, no screening."""
    from oracle import rdm
    out = {}
    for name, P in (("plain", synth.config_plain(0)), ("hubbard4", synth.config_hubbard(4.0))):
        for K in (2, 4, 0):
            t = time.time()
            res = mbe.run(P, max_order=K if K else None)
            gh, ge = rdm.mbe_gradient(P, res)
            key = f"{name}_K{K if K else 'full'}"
            out[key + "_h"] = gh
            out[key + "_eri"] = ge
            out[key + "_E"] = np.array([res.total])
            print(key, f"{time.time() - t:.1f}s", flush=True)
    np.savez_compressed(os.path.join(HERE, "gradients.npz"), **out)
    print("wrote gradients.npz", flush=True)


if __name__ == "__main__":
    which = sys.argv[1:] or ["plain", "hubbard", "sweep", "large", "gradients"]
    for w in which:
        globals()[w]()
