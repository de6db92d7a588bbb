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
  pi_pruned.json       MBE of the plain problem with pi-pruning (a = 0, 5.0)
  screened_weak.json   MBE of a weakly coupled problem whose screening (a = 5.0)
                       removes tuples from order 4 on
  class_samples.json   CASCI energies and the gap to the second root of one or
                       two tuples of every large shape class of the order sweep
                       (also at integral scale std 0.1) and of the 60-orbital
                       problem up to order 4 (dims up to 853776)
  rdm_large.npz        CASCI energy and the active blocks of gamma and Gamma of
                       tuples with 10, 11 and 12 active orbitals
  casscf.json          canonical CASSCF orbitals of [Pi] (energy, U, h) and the
                       full-order MBE in them: plain problem, a 7-orbital
                       problem with a frozen orbital, an open-shell 8-orbital
                       problem, and the plain problem with the singlet
                       reference state and singlet tuple energies
  plain_spin.json      full-order MBE of the plain 10-orbital problem with every
                       CASCI energy that of the tuple's lowest singlet
                       (spin-targeted; the problem's lowest states are often
                       triplets)
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


def pi_pruned():
    """Full-order MBE of the plain 10-orbital problem with pi-pruning over the
    expansion pairs (5, 6) and (7, 8), without screening and with a = 5.0."""
    out = {}
    cache = {}
    for a in (0.0, 5.0):
        P = synth.config_plain(0)
        P.pi_pairs = [(5, 6), (7, 8)]
        P.a = a

        def energy(S):
            if S not in cache:
                cache[S] = fci.casci_energy(P, S)
            return cache[S]
        t = time.time()
        res = mbe.run(P, energy=energy)
        out["a%g" % a] = mbe_json(P, res, {"seconds": time.time() - t})
    out["pairs"] = [[5, 6], [7, 8]]
    out["fci"] = cache[tuple(synth.config_plain(0).expansion_space())]
    write("pi_pruned.json", out)


def screened():
    P = synth.config_weak()
    t = time.time()
    res = mbe.run(P)
    band = []
    for o in res.orders[1:]:
        tau = mbe.screen_threshold(P.a, o.k)
        band += [[o.k, list(tt), d] for tt, d in zip(o.tuples, o.dinc) if abs(abs(d) - tau) < 1e-10]
    write("screened_weak.json", mbe_json(P, res, {"guard_band": band, "seconds": time.time() - t}))


def _eig2(P, S):
    """Lowest two eigenvalues of the CAS of S (oracle Hamiltonian; dense up to
    fci.DENSE_MAX, else ARPACK on the matrix-free product) and the dim."""
    import scipy.sparse.linalg as sla
    sp = fci.cas_space(P, S)
    if sp.dim <= fci.DENSE_MAX:
        w = np.linalg.eigvalsh(fci.hamiltonian_matrix(P, sp))
        return float(w[0]), float(w[1]) if len(w) > 1 else None, sp.dim
    op = sla.LinearOperator((sp.dim, sp.dim), matvec=lambda x: fci.matvec(P, sp, np.asarray(x).reshape(-1)),
                            dtype=np.float64)
    v0 = np.random.default_rng(20190507).standard_normal(sp.dim)
    w = sla.eigsh(op, k=2, which="SA", v0=v0, tol=1e-14, ncv=min(sp.dim - 1, 40), maxiter=100000,
                  return_eigenvectors=False)
    w = np.sort(w)
    return float(w[0]), float(w[1]), sp.dim


# one or two tuples of every large shape class: (problem key, tuple)
CLASS_PICKS = [
    # order sweep, order 4: (8e,10o) 44100, (10e,10o) 63504
    ("sweep", (1, 10, 15, 20)), ("sweep", (1, 2, 11, 19)),
    # order sweep, order 5: (8e,11o) 108900 (4 alpha), (10e,11o) 213444 (5 alpha)
    ("sweep", (1, 9, 14, 18, 23)), ("sweep", (2, 10, 13, 17, 21)),
    ("sweep", (1, 2, 9, 16, 22)), ("sweep", (1, 2, 12, 15, 20)),
    # order sweep with integral scale std 0.1 (20-vector plain scale x 3)
    ("sweep01", ()), ("sweep01", (9,)), ("sweep01", (1,)), ("sweep01", (10, 17)), ("sweep01", (1, 12)),
    ("sweep01", (1, 2)), ("sweep01", (9, 14, 20)), ("sweep01", (2, 11, 16)), ("sweep01", (1, 2, 13)),
    ("sweep01", (11, 13, 18, 21)),
    # 60 orbitals, order 2: (8e,10o) 44100, (10e,10o) 63504, (12e,10o) 44100
    ("large", (10, 35)), ("large", (0, 22)), ("large", (0, 1)),
    # order 4, the dominant classes: (8e,12o) 245025, (10e,12o) 627264, (12e,12o) 853776
    ("large", (10, 25, 40, 55)),
    # order 3: (8e,11o) 108900, (10e,11o) 213444, (12e,11o) 213444
    ("large", (12, 30, 51)), ("large", (1, 20, 44)), ("large", (0, 1, 33)),
    ("large", (0, 11, 29, 47)), ("large", (0, 1, 18, 52)),
]


def _problems():
    return {"sweep": synth.config_sweep(0), "sweep01": synth.config_sweep(0, vec_std=0.1),
            "large": synth.config_large(0)}


def class_samples():
    """Energies and gaps at the large shape classes, written after every tuple."""
    probs = _problems()
    path = os.path.join(HERE, "class_samples.json")
    done = {}
    if os.path.exists(path):
        with open(path) as f:
            for s in json.load(f)["samples"]:
                done[(s["problem"], tuple(s["tuple"]))] = s
    for key, S in CLASS_PICKS:
        if (key, S) in done:
            continue
        t = time.time()
        P = probs[key]
        e0, e1, dim = _eig2(P, S)
        sp = fci.cas_space(P, S)
        done[(key, S)] = {"problem": key, "tuple": list(S), "eps": e0, "eps1": e1, "dim": dim,
                          "n_active": len(sp.active), "na": sp.na, "nb": sp.nb, "seconds": time.time() - t}
        print(key, S, dim, e0, e1, f"{time.time() - t:.1f}s", flush=True)
        write("class_samples.json", {"source": "oracle (fci.cas_space, dense eigvalsh or ARPACK k=2)",
                                     "samples": [done[k] for k in sorted(done, key=lambda k: (k[0], len(k[1]), k[1]))]})


RDM_PICKS = [("sweep", (9, 12, 17, 22)), ("sweep", (13, 16, 20, 22, 23)), ("large", (10, 25, 40, 55))]


def rdm_large():
    """CASCI energy, gap and the active blocks gamma_A [nA, nA], Gamma_A
    [nA, nA, nA, nA] (oracle rdm12 of the ARPACK eigenvector) of tuples with
    10, 11 and 12 active orbitals."""
    from oracle import rdm
    import scipy.sparse.linalg as sla
    probs = _problems()
    out = {}
    for key, S in RDM_PICKS:
        t = time.time()
        P = probs[key]
        sp = fci.cas_space(P, S)
        op = sla.LinearOperator((sp.dim, sp.dim), matvec=lambda x: fci.matvec(P, sp, np.asarray(x).reshape(-1)),
                                dtype=np.float64)
        v0 = np.random.default_rng(20190507).standard_normal(sp.dim)
        w, v = sla.eigsh(op, k=2, which="SA", v0=v0, tol=1e-14, ncv=min(sp.dim - 1, 40), maxiter=100000)
        o = np.argsort(w)
        vec = v[:, o[0]] / np.linalg.norm(v[:, o[0]])
        g1, g2 = rdm.rdm12(P, sp, vec)
        A = np.array(sp.active)
        tag = f"{key}_" + "_".join(map(str, S))
        out[tag + "_eps"] = np.array([w[o[0]], w[o[1]]])
        out[tag + "_active"] = A
        out[tag + "_gamma"] = g1[np.ix_(A, A)]
        out[tag + "_Gamma"] = g2[np.ix_(A, A, A, A)]
        print(tag, sp.dim, w[o[0]], w[o[1]], f"{time.time() - t:.1f}s", flush=True)
        np.savez_compressed(os.path.join(HERE, "rdm_large.npz"), **out)
    print("wrote rdm_large.npz", flush=True)


def casscf():
    """CASSCF expansion references: the canonical CASSCF orbitals of [Pi]
    and the full-order MBE in them, for the plain problem and a 7-orbital
    problem with a frozen orbital."""
    from oracle import casscf as cs
    from oracle import spin
    out = {}
    for key, P, S in (("plain", synth.config_plain(0), None),
                      ("small7", synth.small_problem(7, 3, 3, [2, 3], nfrozen=1, nvec=6, seed=11, vec_std=0.15,
                                                     offdiag_std=0.2), None),
                      ("open8", synth.small_problem(8, 4, 2, [2, 3], nfrozen=1, nvec=6, seed=3, e_const=0.5), None),
                      ("plain_singlet", synth.config_plain(0), 0.0)):
        t0 = time.time()
        # a tight orbital gradient: the tuples' energies are not stationary
        # under orbital rotations, so they follow the orbitals' accuracy
        e, U, Pc = cs.casscf(P, g_tol=1e-11, spin=S)
        if S is None:
            res = mbe.run(Pc, energy=lambda T: fci.casci_energy(Pc, T))
        else:
            res = mbe.run(Pc, energy=lambda T: spin.casci_energy_spin(Pc, T, S))
        out[key] = mbe_json(Pc, res, {"e_casscf": e, "e_casci_start": fci.casci_energy(P, ()),
                                      "h": Pc.h.tolist(), "U": U.tolist(), "spin": S,
                                      "fci": fci.fci_energy(P) if S is None else None,
                                      "seconds": time.time() - t0})
        print(key, e, time.time() - t0, flush=True)
    write("casscf.json", out)


def plain_spin():
    from oracle import spin
    P = synth.config_plain(0)
    t0 = time.time()
    res = mbe.run(P, energy=lambda S: spin.casci_energy_spin(P, S))
    plain_e = {}
    for o in res.orders:
        for S in o.tuples:
            if len(S) <= 2:
                plain_e[",".join(map(str, S))] = fci.casci_energy(P, S)
    write("plain_spin.json", mbe_json(P, res, {"spin": 0, "lowest_any_spin": plain_e,
                                              "seconds": time.time() - t0}))


if __name__ == "__main__":
    which = sys.argv[1:] or ["plain", "hubbard", "sweep", "large", "gradients"]
    for w in which:
        globals()[w]()
