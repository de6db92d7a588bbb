"""Parity of the HIP path (through the C ABI) with the CPU oracle.

Tolerances (FP64 end to end): sigma and the diagonal within 1e-12 relative;
per-tuple CASCI energies within 1e-10 E_h; increments, order sums and totals
within 1e-9 E_h; tuple lists identical."""
import json
import os

import numpy as np
import pytest

import synth
from oracle import fci, mbe as ombe

torch = pytest.importorskip("torch")
import paper_1905_02786_amd as M  # noqa: E402

pytestmark = pytest.mark.gpu
GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


@pytest.fixture(scope="module")
def ws():
    _need_gpu()
    return M.workspace(8 << 30)


def _ctx(P, **opt):
    ctx = M.Context.from_problem(P, device=0, **opt)
    return ctx


def _tuples_with_dims(P, k, limit):
    import itertools
    out = []
    for S in itertools.combinations(P.expansion_space(), k):
        if fci.cas_space(P, S).dim <= limit:
            out.append(S)
    return out


def core_order_signs(sp):
    """Diagonal basis change between the oracle's determinants (creators over
    the full orbital space, ascending, core included) and the library's (core
    creators first, then active alpha, then active beta): reordering gives
    (-1)^(number of pairs (active electron, core orbital) with the electron
    below the core orbital), per spin.  Eigenvalues are unchanged."""
    act = sum(1 << p for p in sp.active)

    def n_below(m):
        return sum(bin(int(m) & act & ((1 << c) - 1)).count("1") for c in sp.core)
    sa = np.array([n_below(m) for m in sp.alist])
    sb = np.array([n_below(m) for m in sp.blist])
    return ((-1.0) ** (sa[:, None] + sb[None, :])).reshape(-1)


PROBLEMS = {
    "plain": lambda: synth.config_plain(0),
    "hubbard4": lambda: synth.config_hubbard(4.0),
    "sweep": lambda: synth.config_sweep(0),
    "large": lambda: synth.config_large(0),
    "openshell": lambda: synth.small_problem(8, 4, 2, [2, 3], nfrozen=1, nvec=6, seed=3, e_const=0.5),
}

SIGMA_CASES = [
    ("plain", ()), ("plain", (0,)), ("plain", (5,)), ("plain", (0, 9)), ("plain", (2, 5, 6)),
    ("plain", (0, 1, 5, 6)), ("plain", (0, 1, 2, 5, 6, 7)),
    ("hubbard4", (2, 7)), ("hubbard4", (0, 1, 6, 7, 8)),
    ("sweep", ()), ("sweep", (1,)), ("sweep", (9, 13)), ("sweep", (1, 2, 10)),
    ("sweep", (9, 10, 11, 12, 13)), ("large", (10, 11)),
    ("openshell", ()), ("openshell", (1, 5)), ("openshell", (1, 4, 5, 6, 7)),
    # the order sweep's largest classes: n_A = 11 with 4 and 5 alpha electrons
    ("sweep", (1, 9, 10, 11, 12)), ("sweep", (1, 2, 9, 10, 11)),
    # the 60-orbital problem at n_A = 12: (8e,12o), (10e,12o), (12e,12o), and n_A = 13
    ("large", (10, 11, 12, 13)), ("large", (0, 10, 11, 12)), ("large", (0, 1, 10, 11)),
    ("large", (10, 11, 12, 13, 14)),
]

_PROBLEM_CACHE = {}
_REF_CACHE = {}


def _problem(name):
    if name not in _PROBLEM_CACHE:
        _PROBLEM_CACHE[name] = PROBLEMS[name]()
    return _PROBLEM_CACHE[name]


def _sigma_reference(name, S):
    """Oracle sigma of seeded vectors (one above 200000 determinants) in the
    library's determinant signs, and the oracle diagonal where it is dense;
    computed once per case and shared by the variants."""
    key = (name, S)
    if key not in _REF_CACHE:
        P = _problem(name)
        sp = fci.cas_space(P, S)
        rng = np.random.default_rng(sum(S) + 7)
        print(f"oracle sigma {name} {S} dim {sp.dim} ...", flush=True)
        c = rng.standard_normal((2 if sp.dim <= 200000 else 1, sp.dim))
        sg = core_order_signs(sp)
        if sp.dim <= 2000:
            H = fci.hamiltonian_matrix(P, sp)
            ref = sg * ((sg * c) @ H.T)
            ref_diag = np.diag(H)
        else:
            ref = np.stack([sg * fci.matvec(P, sp, sg * v) for v in c])
            # sampled diagonal elements <I|H|I> (Slater-Condon, E_const included)
            from oracle import native
            L = native.lib()
            h = np.ascontiguousarray(P.h)
            eri = np.ascontiguousarray(P.eri)
            ref_diag = {}
            for I in rng.choice(sp.dim, size=6, replace=False):
                a, b = int(sp.alist[I // len(sp.blist)]), int(sp.blist[I % len(sp.blist)])
                ref_diag[int(I)] = P.e_const + L.sc_element(P.norb, native.ptr(h), native.ptr(eri), a, b, a, b)
        _REF_CACHE[key] = (sp, c, ref, ref_diag)
    return _REF_CACHE[key]


# (sigma_variant, linked_rows): column strip with linked rows where n_A >= 9
# (the default), column strip on all pair rows, linked rows wherever they fit
# with the A rows gathered (2) or resident in LDS (3), the form with the
# diagonal sums on the vector ALU wherever it fits (4), the linked rows
# through W in the workspace wherever it fits (5), materialised W
@pytest.mark.parametrize("variant,linked", [(1, 1), (1, 0), (1, 2), (1, 3), (1, 4), (1, 5), (2, 1)])
@pytest.mark.parametrize("name,S", SIGMA_CASES)
def test_hdiag_and_sigma_match_oracle(ws, name, S, variant, linked):
    P = _problem(name)
    ctx = _ctx(P, sigma_variant=variant, linked_rows=linked)
    sp, c, ref, ref_diag = _sigma_reference(name, S)
    print(f"case {name} {S} dim {sp.dim} variant {variant} linked {linked}", flush=True)
    ct = torch.tensor(c, device="cuda:0")
    sig = ctx.tuple_sigma(len(S), S, ct, ws).cpu().numpy()
    scale = max(1.0, np.abs(ref).max())
    assert np.abs(sig - ref).max() <= 1e-12 * scale, np.abs(sig - ref).max()
    hd = ctx.tuple_hdiag(len(S), S, ws).cpu().numpy()
    if isinstance(ref_diag, dict):
        # sampled determinants
        for I, v in ref_diag.items():
            assert abs(hd[I] - v) <= 1e-12 * max(1.0, abs(v))
    else:
        assert np.abs(hd - ref_diag).max() <= 1e-12 * max(1.0, np.abs(ref_diag).max())


def test_sigma_is_symmetric_full_space(ws):
    P = synth.config_plain(0)
    S = tuple(P.expansion_space())
    ctx = _ctx(P)
    sh = ctx.tuple_shape(len(S), S)
    assert sh["dim"] == 44100
    rng = np.random.default_rng(3)
    x = torch.tensor(rng.standard_normal((2, sh["dim"])), device="cuda:0")
    sx = ctx.tuple_sigma(len(S), S, x, ws)
    a = float(torch.dot(x[0], sx[1]))
    b = float(torch.dot(sx[0], x[1]))
    assert abs(a - b) <= 1e-12 * max(abs(a), 1.0)


def test_energies_orders_0_to_3_match_oracle(ws):
    P = synth.config_plain(0)
    ctx = _ctx(P)
    for k in range(0, 4):
        tuples = _tuples_with_dims(P, k, 10 ** 9) if k else [()]
        e, st = ctx.solve_tuples(k, tuples if k else [()], ws)
        assert (st == 0).all()
        ref = np.array([fci.casci_energy(P, S) for S in tuples])
        print(f"order {k}: {len(tuples)} tuples, max |dE| = {np.abs(e - ref).max():.2e}", flush=True)
        assert np.abs(e - ref).max() <= 1e-10


@pytest.mark.parametrize("variant", [1, 2])
def test_batched_and_per_solve_agree_bitwise(ws, variant):
    P = synth.config_plain(0)
    tuples = _tuples_with_dims(P, 2, 10 ** 9)
    e1, s1 = _ctx(P, batched=1, sigma_variant=variant).solve_tuples(2, tuples, ws)
    e0, s0 = _ctx(P, batched=0, sigma_variant=variant).solve_tuples(2, tuples, ws)
    assert (s1 == 0).all() and (s0 == 0).all()
    assert np.array_equal(e1, e0)


def test_sigma_variants_agree(ws):
    """The column-strip and materialised-W sigma give the same energies."""
    P = synth.config_sweep(0)
    import itertools
    tuples = list(itertools.combinations(P.expansion_space(), 3))[::7]
    e1, s1 = _ctx(P, sigma_variant=1).solve_tuples(3, tuples, ws)
    e2, s2 = _ctx(P, sigma_variant=2).solve_tuples(3, tuples, ws)
    assert (s1 == 0).all() and (s2 == 0).all()
    assert np.abs(e1 - e2).max() <= 1e-10


def test_linked_rows_solves(ws):
    """Order-5 tuples of the 24-orbital sweep (n_A = 11, the linked-row strip
    kernel): a repeat run and the per-solve path give bitwise the same
    energies, and the all-pairs strip kernel the same within 1e-10."""
    P = synth.config_sweep(0)
    import itertools
    tuples = list(itertools.combinations(P.expansion_space(), 5))[::1500][:4]
    ctx = _ctx(P)
    assert all(ctx.tuple_shape(5, S)["n_active"] == 11 for S in tuples)
    e1, s1 = ctx.solve_tuples(5, tuples, ws)
    e2, s2 = _ctx(P).solve_tuples(5, tuples, ws)
    e3, s3 = _ctx(P, batched=0).solve_tuples(5, tuples, ws)
    e4, s4 = _ctx(P, linked_rows=0).solve_tuples(5, tuples, ws)
    assert all((s == 0).all() for s in (s1, s2, s3, s4))
    assert np.array_equal(e1, e2) and np.array_equal(e1, e3)
    assert np.abs(e1 - e4).max() <= 1e-10


def test_repeat_runs_are_bitwise_identical(ws):
    P = synth.config_hubbard(8.0)
    tuples = _tuples_with_dims(P, 3, 10 ** 9)
    ctx = _ctx(P)
    e1, _ = ctx.solve_tuples(3, tuples, ws)
    e2, _ = ctx.solve_tuples(3, tuples, ws)
    assert np.array_equal(e1, e2)


def _check_against_golden(res, g, tol_eps=1e-10, tol_inc=1e-9):
    assert len(res.orders) == len(g["orders"])
    for o, go in zip(res.orders, g["orders"]):
        assert [list(map(int, t)) for t in o.tuples] == [list(t) for t in go["tuples"]] or o.k == 0
        assert (o.status == 0).all()
        assert np.abs(o.eps - np.array(go["eps"])).max() <= tol_eps, o.k
        assert np.abs(o.dinc - np.array(go["dinc"])).max() <= tol_inc, o.k
        assert abs(o.order_sum - go["order_sum"]) <= tol_inc
    assert abs(res.total - g["total"]) <= tol_inc


def test_plain_full_order_mbe_equals_fci(ws):
    with open(os.path.join(GOLDEN, "plain_s0.json")) as f:
        g = json.load(f)
    P = synth.config_plain(0)
    res = _ctx(P).run(ws)
    _check_against_golden(res, g)
    assert abs(res.total - g["fci"]) <= 1e-9
    assert [len(o.tuples) for o in res.orders] == [1, 8, 28, 56, 70, 56, 28, 8, 1]


@pytest.mark.parametrize("U", [2.0, 4.0, 8.0])
def test_hubbard_chain_mbe(ws, U):
    with open(os.path.join(GOLDEN, f"hubbard_U{U:g}.json")) as f:
        g = json.load(f)
    P0 = synth.config_hubbard(U)
    res0 = _ctx(P0).run(ws)
    _check_against_golden(res0, g["unscreened"])
    assert abs(res0.total - g["fci"]) <= 1e-9
    P5 = synth.config_hubbard(U, a=5.0)
    res5 = _ctx(P5).run(ws)
    _check_against_golden(res5, g["screened"])


def _solve_samples(P, fname, ws):
    path = os.path.join(GOLDEN, fname)
    if not os.path.exists(path):
        pytest.skip(f"{fname} not generated")
    with open(path) as f:
        g = json.load(f)
    ctx = _ctx(P)
    worst = 0.0
    for smp in g["samples"]:
        S = tuple(smp["tuple"])
        e, st = ctx.solve_tuples(len(S), [S] if S else [()], ws)
        assert st[0] == 0
        worst = max(worst, abs(e[0] - smp["eps"]))
        assert abs(e[0] - smp["eps"]) <= 1e-10, (S, e[0], smp["eps"])
    print(f"{fname}: {len(g['samples'])} samples, max |dE| = {worst:.2e}")


# Tuples spanning P spaces smaller than, equal to and larger than the CAS
# (dims 1 ... 1225), on the strongly correlated Hubbard chain and the open-shell
# problem; the U/t = 8 order-5 tuple is the hardest case for the P-space
# preconditioner.
PSPACE_CASES = [
    ("hubbard8", (1, 2, 3, 6, 9)), ("hubbard8", (0, 2, 6)), ("hubbard8", (0,)), ("hubbard8", ()),
    ("hubbard8", (0, 1, 2, 6)), ("openshell", ()), ("openshell", (1,)), ("openshell", (1, 4, 5, 6, 7)),
]


@pytest.mark.parametrize("pspace", [0, 1, 7, 128])
def test_pspace_settings_match_oracle(ws, pspace):
    """With the P-space preconditioner some corrections lie mostly inside the
    subspace and take the two explicit Gram-Schmidt passes instead of joining
    the basis through the triangular factor: with P spaces of 7 and 128 these
    cases go through that path too (counted in the stats).  The batched
    iteration (whole-tuple mode off; that mode's settings are covered in
    test_gpu_whole.py)."""
    probs = {"hubbard8": synth.config_hubbard(8.0), "openshell": PROBLEMS["openshell"]()}
    worst = 0.0
    second = 0
    for name, S in PSPACE_CASES:
        P = probs[name]
        ctx = _ctx(P, pspace=pspace, whole_dim=0)
        e, st = ctx.solve_tuples(len(S), [S] if S else [()], ws)
        second += ctx.stats()["gs_second_pass"]
        e_ref = fci.casci_energy(P, S)
        assert st[0] == 0, (name, S, pspace, st[0])
        assert abs(e[0] - e_ref) <= 1e-10, (name, S, pspace, e[0], e_ref)
        worst = max(worst, abs(e[0] - e_ref))
    print(f"pspace {pspace}: max |dE| = {worst:.1e}, {second} corrections with two explicit passes")
    if pspace >= 7:
        assert second > 0


@pytest.mark.parametrize("max_space", [2, 3, 4, 20, 32])
def test_max_space_settings_match_oracle(ws, max_space):
    """Subspace bounds other than the default: a restart after every one or two
    expansions (2, 3: the correction goes to basis slot 1 and the triangular
    factor restarts from the Ritz vector), frequent restarts (4) and the
    32-vector kernel instantiations, on odd and even dimensions."""
    probs = {"hubbard8": synth.config_hubbard(8.0), "sweep": synth.config_sweep(0)}
    cases = [("hubbard8", (1, 2, 3, 6, 9)), ("hubbard8", (0, 1, 2, 6)), ("hubbard8", (0, 2, 6, 8)),
             ("sweep", (1,)), ("sweep", (9, 18))]
    worst = 0.0
    for name, S in cases:
        P = probs[name]
        ctx = _ctx(P, max_space=max_space, max_iter=1000)
        e, st = ctx.solve_tuples(len(S), [S], ws)
        e_ref = fci.casci_energy(P, S)
        assert st[0] == 0, (name, S, max_space, st[0])
        assert abs(e[0] - e_ref) <= 1e-10, (name, S, max_space, e[0], e_ref)
        worst = max(worst, abs(e[0] - e_ref))
    print(f"max_space {max_space}: max |dE| = {worst:.1e}")


def test_sweep_sampled_tuples(ws):
    _solve_samples(synth.config_sweep(0), "sweep_sample.json", ws)


def test_large_sampled_tuples(ws):
    _solve_samples(synth.config_large(0), "large_sample.json", ws)


def test_screened_sweep_lists_match_oracle_assembler(ws):
    """Orders 1-3 of the 24-orbital sweep with a = 5.0: the oracle's own
    assembler and screening, fed the GPU energies, reproduce the GPU's tuple
    lists and increments exactly."""
    P = synth.config_sweep(0, max_order=3)
    res = _ctx(P).run(ws)
    table = {}
    for o in res.orders:
        for t, e in zip(o.tuples, o.eps):
            table[tuple(int(x) for x in t)] = float(e)
    ref = ombe.run(P, energy=lambda S: table[tuple(S)])
    for o, ro in zip(res.orders, ref.orders):
        assert [tuple(int(x) for x in t) for t in o.tuples] == list(ro.tuples)
        assert np.array_equal(o.dinc, np.array(ro.dinc))


def test_edge_cases(ws):
    # single-determinant CAS: RHF reference space, order 0
    P = synth.small_problem(6, 2, 2, [0, 1], nvec=4, seed=2)
    ctx = _ctx(P)
    assert ctx.tuple_shape(0, ())["dim"] == 1
    e, st = ctx.solve_tuples(0, [()], ws)
    assert st[0] == 0 and abs(e[0] - fci.casci_energy(P, ())) <= 1e-12
    # empty tuple list
    e, st = ctx.solve_tuples(1, np.zeros((0, 1), np.int16), ws)
    assert e.shape == (0,)
    # a one-tuple workspace that is too small
    with pytest.raises(M.MBEFCIError) as ex:
        ctx.solve_tuples(1, [(3,)], ws[:1024])
    assert ex.value.code == -2
    # out-of-space tuple
    with pytest.raises(M.MBEFCIError):
        ctx.solve_tuples(1, [(0,)], ws)
    # one electron
    P1 = synth.small_problem(5, 1, 0, [0], nvec=3, seed=1)
    e, st = _ctx(P1).solve_tuples(4, [(1, 2, 3, 4)], ws)
    assert abs(e[0] - fci.casci_energy(P1, (1, 2, 3, 4))) <= 1e-10


def test_screening_removes_tuples_on_device(ws):
    """A weakly coupled problem on which a = 5.0 screens out 5 of the 35
    order-4 candidates and 11 of the 21 order-5 ones: the device run, with its
    own energies, takes the same screening decisions as the oracle run with
    the oracle's energies (identical lists), and every |d_eps| within 1e-10 of
    its threshold (the guard band) is reported; the stored run has none."""
    with open(os.path.join(GOLDEN, "screened_weak.json")) as f:
        g = json.load(f)
    P = synth.config_weak()
    res = _ctx(P).run(ws)
    counts = [len(o.tuples) for o in res.orders]
    assert counts == [len(o["tuples"]) for o in g["orders"]] == [1, 7, 21, 35, 30, 10]
    _check_against_golden(res, g)
    band = []
    for o in res.orders[1:]:
        tau = ombe.screen_threshold(P.a, o.k)
        band += [(o.k, tuple(int(x) for x in t), float(d)) for t, d in zip(o.tuples, o.dinc)
                 if abs(abs(d) - tau) < 1e-10]
    print(f"screened counts {counts}; device guard band {band}; stored guard band {g['guard_band']}")
    assert not band and not g["guard_band"]


@pytest.mark.parametrize("a", [0.0, 5.0])
def test_pi_pruned_mbe_matches_oracle(ws, a):
    """Pi-pruning on the device run (pairs (5, 6), (7, 8) of the plain problem):
    the tuple lists, energies, increments and sums of the oracle's run, and at
    full order still the FCI energy (Eq. 3 telescopes over any computed set
    that contains the top tuple)."""
    path = os.path.join(GOLDEN, "pi_pruned.json")
    if not os.path.exists(path):
        pytest.skip("pi_pruned.json not generated")
    with open(path) as f:
        g = json.load(f)
    P = synth.config_plain(0)
    P.pi_pairs = [tuple(p) for p in g["pairs"]]
    P.a = a
    res = _ctx(P).run(ws)
    _check_against_golden(res, g["a%g" % a])
    print(f"a = {a}: counts {[len(o.tuples) for o in res.orders]}")
    assert abs(res.total - g["fci"]) <= 1e-9


def test_iteration_blocks_and_graphs_give_the_same_energies(ws):
    """Davidson iterations launched one per host round trip (profile = 1), in
    blocks (graph = 0) and as a replayed hipGraph (graph = 1): the same
    arithmetic, so bitwise the same energies, on tuples that take the
    explicit Gram-Schmidt passes too (Hubbard U/t = 8, P space 7; the
    whole-tuple mode, which would take these small classes, off)."""
    P = synth.config_hubbard(8.0)
    tuples = _tuples_with_dims(P, 4, 10 ** 9)
    out = []
    for opts in (dict(profile=1), dict(profile=0, graph=0), dict(profile=0, graph=1)):
        ctx = _ctx(P, pspace=7, whole_dim=0, **opts)
        e, st = ctx.solve_tuples(4, tuples, ws)
        assert (st == 0).all()
        out.append(e)
        if opts.get("graph") == 1:
            assert ctx.stats()["graph_batches"] > 0
    assert np.array_equal(out[0], out[1]) and np.array_equal(out[0], out[2])
    ref = np.array([fci.casci_energy(P, S) for S in tuples[:6]])
    assert np.abs(out[2][:6] - ref).max() <= 1e-10


def test_autotuned_forms_match_oracle(ws):
    """The autotuner's choice of sigma form and GEMM tile (order-4 tuples of
    the order sweep, 14400-63504 determinants) gives the energies of the fixed
    default forms within 1e-10 and of the oracle's stored samples."""
    P = synth.config_sweep(0)
    import itertools
    tuples = list(itertools.combinations(P.expansion_space(), 4))[::97]
    ctx = _ctx(P, autotune=1)
    e1, s1 = ctx.solve_tuples(4, tuples, ws)
    e0, s0 = _ctx(P, autotune=0).solve_tuples(4, tuples, ws)
    assert (s1 == 0).all() and (s0 == 0).all()
    assert np.abs(e1 - e0).max() <= 1e-10
    e2, _ = ctx.solve_tuples(4, tuples, ws)       # the choice is kept: bitwise repeat
    assert np.array_equal(e1, e2)
