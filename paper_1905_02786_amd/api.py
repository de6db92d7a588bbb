"""Thin Python binding of libmbefci.so (argument marshalling only).

Every step of the MBE-FCI path (tuple generation, screening, integral gather,
Hamiltonian diagonal, sigma, Davidson, increment assembly) runs inside the
library; PyTorch provides the device workspace and the stream.
"""
from __future__ import annotations

import ctypes
from dataclasses import dataclass, field

import numpy as np

from . import _lib

STATUS_NAMES = {0: "OK", -1: "EINVAL", -2: "ENOMEM", -3: "EDEVICE", -4: "ENOCONV", -5: "ESTATE",
                -6: "ETOOLARGE"}
TUPLE_OK, TUPLE_MAXITER, TUPLE_NONFINITE, TUPLE_STALLED, TUPLE_PENDING = 0, 1, 2, 3, 4


class MBEFCIError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{STATUS_NAMES.get(code, code)}: {msg}")
        self.code = code


def _p(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def default_options() -> _lib.Options:
    o = _lib.Options()
    _lib.load().mbefci_default_options(ctypes.byref(o))
    return o


@dataclass
class Order:
    k: int
    tuples: np.ndarray          # int16 [ntup, k]
    eps: np.ndarray             # float64 [ntup]
    dinc: np.ndarray            # float64 [ntup]
    status: np.ndarray          # int32 [ntup]
    order_sum: float
    wall_ms: float


@dataclass
class Result:
    orders: list = field(default_factory=list)
    total: float = 0.0
    e_base: float = 0.0   # base energy of the whole space (options.base_model)

    def tuple_lists(self):
        return [[tuple(int(x) for x in row) for row in o.tuples] for o in self.orders]


def _read_result(L, res) -> Result:
    out = Result()
    n = L.mbefci_result_norders(res)
    for k in range(n):
        nt = ctypes.c_int64()
        tp, ep, dp, sp = ctypes.c_void_p(), ctypes.c_void_p(), ctypes.c_void_p(), ctypes.c_void_p()
        osum, wall = ctypes.c_double(), ctypes.c_double()
        rc = L.mbefci_result_order(res, k, ctypes.byref(nt), ctypes.byref(tp), ctypes.byref(ep),
                                   ctypes.byref(dp), ctypes.byref(sp), ctypes.byref(osum), ctypes.byref(wall))
        if rc != 0:
            raise MBEFCIError(rc, "result_order")
        m = nt.value
        if m == 0:   # an empty order (pi-pruning)
            out.orders.append(Order(k, np.zeros((0, k), dtype=np.int16), np.zeros(0), np.zeros(0),
                                    np.zeros(0, dtype=np.int32), osum.value, wall.value))
            continue
        if k > 0:
            tb = ctypes.string_at(tp.value, 2 * m * k)
            tuples = np.frombuffer(tb, dtype=np.int16).reshape(m, k).copy()
        else:
            tuples = np.zeros((1, 0), dtype=np.int16)
        eps = np.frombuffer(ctypes.string_at(ep.value, 8 * m), dtype=np.float64).copy()
        dinc = np.frombuffer(ctypes.string_at(dp.value, 8 * m), dtype=np.float64).copy()
        st = np.frombuffer(ctypes.string_at(sp.value, 4 * m), dtype=np.int32).copy()
        out.orders.append(Order(k, tuples, eps, dinc, st, osum.value, wall.value))
    out.total = L.mbefci_result_total(res)
    out.e_base = L.mbefci_result_base(res)
    return out


class Context:
    """One library context: a Hamiltonian, the orbital spaces and options.

    device = None creates a host-only context (planner only, no GPU)."""

    def __init__(self, device: int | None = 0, stream=None):
        self.L = _lib.load()
        self.ptr = ctypes.c_void_p()
        self.device = device
        if device is None:
            rc = self.L.mbefci_create(ctypes.byref(self.ptr), -1, None)
        else:
            if stream is None:
                import torch
                stream = torch.cuda.current_stream(device).cuda_stream
            rc = self.L.mbefci_create(ctypes.byref(self.ptr), int(device), ctypes.c_void_p(stream))
        if rc != 0:
            raise MBEFCIError(rc, "mbefci_create failed")
        self._keep = []

    def __del__(self):
        try:
            if self.ptr:
                self.L.mbefci_destroy(self.ptr)
                self.ptr = ctypes.c_void_p()
        except Exception:
            pass

    def _check(self, rc, allow=()):
        if rc != 0 and rc not in allow:
            raise MBEFCIError(rc, (self.L.mbefci_last_error(self.ptr) or b"").decode())
        return rc

    # -- inputs ---------------------------------------------------------------
    def set_hamiltonian(self, h, eri, e_const=0.0):
        h = np.ascontiguousarray(h, dtype=np.float64)
        eri = np.ascontiguousarray(eri, dtype=np.float64)
        n = h.shape[0]
        if eri.size == n ** 4:
            layout = 0
        else:
            layout = 1
        self._check(self.L.mbefci_set_hamiltonian(self.ptr, n, _p(h), _p(eri), layout, float(e_const)))
        self.norb = n
        self.eri_layout = layout

    def set_spaces(self, nalpha, nbeta, nfrozen, ref):
        r = np.ascontiguousarray(list(ref), dtype=np.int32)
        self._check(self.L.mbefci_set_spaces(self.ptr, int(nalpha), int(nbeta), int(nfrozen),
                                             _p(r) if r.size else None, int(r.size)))

    def set_pi_pairs(self, pairs):
        """Pi-pruning: pairs of expansion orbitals entering tuples together."""
        a = np.ascontiguousarray(np.asarray(list(pairs), dtype=np.int32).reshape(-1))
        self._check(self.L.mbefci_set_pi_pairs(self.ptr, _p(a) if a.size else None, int(a.size // 2)))

    def set_orbital_irreps(self, labels):
        """Abelian irrep labels (0..7) of the orbitals, for options
        sym_shift / irrep (states of a given spatial symmetry)."""
        lab = np.ascontiguousarray(labels, dtype=np.int32)
        self._check(self.L.mbefci_set_orbital_irreps(self.ptr, _p(lab)))

    def set_options(self, **kw):
        o = default_options()
        for k, v in kw.items():
            if not hasattr(o, k):
                raise KeyError(k)
            setattr(o, k, v)
        self._check(self.L.mbefci_set_options(self.ptr, ctypes.byref(o)))
        self.options = o

    @classmethod
    def from_problem(cls, problem, device=0, stream=None, **options):
        ctx = cls(device, stream)
        ctx.set_hamiltonian(problem.h, problem.eri, problem.e_const)
        ctx.set_spaces(problem.nalpha, problem.nbeta, problem.nfrozen, problem.ref)
        if getattr(problem, "pi_pairs", None):
            ctx.set_pi_pairs(problem.pi_pairs)
        opts = dict(a=problem.a, max_order=problem.max_order)
        opts.update(options)
        ctx.set_options(**opts)
        return ctx

    # -- solves ---------------------------------------------------------------
    @staticmethod
    def _tuples(order, tuples):
        t = np.ascontiguousarray(np.asarray(tuples, dtype=np.int16).reshape(-1, order) if order > 0
                                 else np.zeros((len(tuples) if hasattr(tuples, "__len__") else 1, 0), np.int16))
        return t

    def workspace_query(self, order, tuples):
        t = self._tuples(order, tuples)
        mn, want = ctypes.c_size_t(), ctypes.c_size_t()
        self._check(self.L.mbefci_workspace_query(self.ptr, order, t.shape[0], _p(t) if t.size else None,
                                                  ctypes.byref(mn), ctypes.byref(want)))
        return mn.value, want.value

    def solve_tuples(self, order, tuples, workspace, allow_noconv=False):
        """eps(S) for each tuple row; workspace: a torch uint8 CUDA tensor."""
        t = self._tuples(order, tuples)
        n = t.shape[0]
        if not getattr(workspace, "is_cuda", False):
            raise ValueError("workspace must be a CUDA tensor")
        e = np.zeros(n)
        st = np.zeros(n, dtype=np.int32)
        rc = self.L.mbefci_solve_tuples(self.ptr, order, n, _p(t) if t.size else None,
                                        ctypes.c_void_p(workspace.data_ptr()), workspace.numel(), _p(e), _p(st))
        self._check(rc, allow=(-4,) if allow_noconv else ())
        return e, st

    def solve_tuples_noalloc(self, order, tuples, allow_noconv=False):
        """eps(S) for each tuple row with the library's static device workspace
        (no device allocation; calls on one GPU must not overlap)."""
        t = self._tuples(order, tuples)
        n = t.shape[0]
        e = np.zeros(n)
        st = np.zeros(n, dtype=np.int32)
        rc = self.L.mbefci_solve_tuples_noalloc(self.ptr, order, n, _p(t) if t.size else None, _p(e), _p(st))
        self._check(rc, allow=(-4,) if allow_noconv else ())
        return e, st

    def run(self, workspace, allow_noconv=False, keep=False):
        """The whole expansion.  keep=True returns (Result, ResultHandle) so
        that backward() can use the library's copy of the tuple set."""
        if not getattr(workspace, "is_cuda", False):
            raise ValueError("workspace must be a CUDA tensor")
        res = ctypes.c_void_p()
        rc = self.L.mbefci_run(self.ptr, ctypes.c_void_p(workspace.data_ptr()), workspace.numel(),
                               ctypes.byref(res))
        self._check(rc, allow=(-4,) if allow_noconv else ())
        out = _read_result(self.L, res)
        if keep:
            return out, ResultHandle(self.L, res)
        self.L.mbefci_result_free(res)
        return out

    def order_solve(self, handle, first, stride, count, workspace, allow_noconv=False):
        """Solve tuples first + i * stride (i < count) of the open (streamed)
        last order of `handle` (a run with stream_last = 1)."""
        rc = self.L.mbefci_order_solve(self.ptr, handle.ptr, int(first), int(stride), int(count),
                                       ctypes.c_void_p(workspace.data_ptr()), workspace.numel())
        return self._check(rc, allow=(-4,) if allow_noconv else ())

    def order_close(self, handle, allow_noconv=False):
        """Close the streamed order (every tuple solved) and return the Result."""
        rc = self.L.mbefci_order_close(self.ptr, handle.ptr)
        self._check(rc, allow=(-4,) if allow_noconv else ())
        return _read_result(self.L, handle.ptr)

    def result(self, handle) -> Result:
        return _read_result(self.L, handle.ptr)

    def backward(self, handle, workspace, gE=1.0):
        """(dE/dh1 [n, n], dE/d(pq|rs)) of the summed MBE energy, times gE,
        with the tuple set of `handle` held fixed; dE/d(pq|rs) is [n, n, n, n]
        or, for packed integrals, the packed vector (orbit sums)."""
        n = self.norb
        gh = np.zeros((n, n))
        if self.eri_layout == 0:
            ge = np.zeros((n, n, n, n))
        else:
            npair = n * (n + 1) // 2
            ge = np.zeros(npair * (npair + 1) // 2)
        self._check(self.L.mbefci_backward(self.ptr, handle.ptr, float(gE), ctypes.c_void_p(workspace.data_ptr()),
                                           workspace.numel(), _p(gh), _p(ge)))
        return gh, ge

    def tuple_rdm(self, order, tuple_, workspace):
        """(energy, gamma [n, n], Gamma [n, n, n, n]) of one tuple's CASCI
        ground state, frozen core included."""
        n = self.norb
        t = self._tuples(order, [tuple_] if order > 0 else [()])
        e = ctypes.c_double()
        g1 = np.zeros((n, n))
        g2 = np.zeros((n, n, n, n))
        self._check(self.L.mbefci_tuple_rdm(self.ptr, order, _p(t) if t.size else None,
                                            ctypes.c_void_p(workspace.data_ptr()), workspace.numel(),
                                            ctypes.byref(e), _p(g1), _p(g2)))
        return e.value, g1, g2

    def casscf(self, workspace, max_iter: int = 500, g_tol: float = 1e-10) -> dict:
        """CASSCF orbitals of the reference space; the context's Hamiltonian
        is replaced by the one in the canonical CASSCF orbitals.  Returns
        {"energy", "U" [n, n] (columns: new orbitals), "iterations"}."""
        n = self.norb
        U = np.zeros((n, n))
        e = ctypes.c_double()
        it = ctypes.c_int32()
        self._check(self.L.mbefci_casscf(self.ptr, ctypes.c_void_p(workspace.data_ptr()), workspace.numel(),
                                         int(max_iter), float(g_tol), _p(U), ctypes.byref(e), ctypes.byref(it)))
        return {"energy": e.value, "U": U, "iterations": it.value}

    def hf(self, workspace, max_iter: int = 2000, g_tol: float = 1e-10) -> dict:
        """Restricted closed-shell Hartree-Fock orbitals; the context's
        Hamiltonian is replaced by the one in the canonical HF orbitals.
        Returns {"energy", "U" [n, n] (columns: new orbitals), "iterations"}."""
        n = self.norb
        U = np.zeros((n, n))
        e = ctypes.c_double()
        it = ctypes.c_int32()
        self._check(self.L.mbefci_hf(self.ptr, ctypes.c_void_p(workspace.data_ptr()), workspace.numel(),
                                     int(max_iter), float(g_tol), _p(U), ctypes.byref(e), ctypes.byref(it)))
        return {"energy": e.value, "U": U, "iterations": it.value}

    def tuple_base(self, order, tuples, workspace):
        """Base-model energies eps_base of a list of tuples of one order, of
        the model options.base_model names: 1 second order, 2 CCSD, 3 CCSD(T)
        (0 gives the second-order one)."""
        tl = list(tuples) if order > 0 else [()]
        t = self._tuples(order, tl)
        out = np.zeros(len(tl))
        self._check(self.L.mbefci_tuple_base(self.ptr, order, len(tl), _p(t) if t.size else None,
                                             ctypes.c_void_p(workspace.data_ptr()), workspace.numel(), _p(out)))
        return out

    def hamiltonian(self):
        """(h [n, n], (pq|rs) [n, n, n, n], constant) of the context."""
        n = self.norb
        h = np.zeros((n, n))
        eri = np.zeros((n, n, n, n))
        c = ctypes.c_double()
        self._check(self.L.mbefci_get_hamiltonian(self.ptr, _p(h), _p(eri), ctypes.byref(c)))
        return h, eri, c.value

    def run_host(self, energy) -> Result:
        """The planner with tuple energies from the Python callable
        energy(order, tuples[int16 ntup x order]) -> float64 array."""
        err = []

        def cb(user, order, ntup, tuples, out):
            try:
                if order > 0:
                    arr = np.ctypeslib.as_array(tuples, shape=(ntup * order,)).reshape(ntup, order).copy()
                else:
                    arr = np.zeros((ntup, 0), dtype=np.int16)
                e = np.asarray(energy(order, arr), dtype=np.float64)
                for i in range(ntup):
                    out[i] = float(e[i])
                return 0
            except Exception as ex:  # pragma: no cover - surfaced below
                err.append(ex)
                return 1

        fn = _lib.ENERGY_FN(cb)
        res = ctypes.c_void_p()
        rc = self.L.mbefci_run_host(self.ptr, fn, None, ctypes.byref(res))
        if err:
            raise err[0]
        self._check(rc)
        try:
            return _read_result(self.L, res)
        finally:
            self.L.mbefci_result_free(res)

    # -- single tuple kernels -------------------------------------------------
    def tuple_shape(self, order, tuple_):
        t = self._tuples(order, [tuple_] if order > 0 else [()])
        na, nb = ctypes.c_int64(), ctypes.c_int64()
        nact, naa, nba = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
        self._check(self.L.mbefci_tuple_shape(self.ptr, order, _p(t) if t.size else None, ctypes.byref(na),
                                              ctypes.byref(nb), ctypes.byref(nact), ctypes.byref(naa),
                                              ctypes.byref(nba)))
        return dict(n_alpha_strings=na.value, n_beta_strings=nb.value, dim=na.value * nb.value,
                    n_active=nact.value, n_alpha_active=naa.value, n_beta_active=nba.value)

    def tuple_sigma(self, order, tuple_, c, workspace, out=None):
        """sigma = H c on the device for vectors c [nvec, dim] (torch float64 CUDA)."""
        import torch
        t = self._tuples(order, [tuple_] if order > 0 else [()])
        dim = self.tuple_shape(order, tuple_)["dim"]
        c = c.contiguous()
        if c.dtype != torch.float64 or not c.is_cuda or c.numel() % dim or c.numel() == 0:
            raise ValueError(f"c must be a non-empty float64 CUDA tensor of nvec x {dim} elements")
        nvec = c.numel() // dim
        if out is None:
            out = torch.empty_like(c)
        if out.shape != c.shape or out.dtype != torch.float64 or not out.is_contiguous():
            raise ValueError("out must match c")
        self._check(self.L.mbefci_tuple_sigma(self.ptr, order, _p(t) if t.size else None,
                                              ctypes.c_void_p(workspace.data_ptr()), workspace.numel(),
                                              ctypes.c_void_p(c.data_ptr()), ctypes.c_void_p(out.data_ptr()),
                                              nvec))
        return out

    def tuple_hdiag(self, order, tuple_, workspace):
        import torch
        sh = self.tuple_shape(order, tuple_)
        t = self._tuples(order, [tuple_] if order > 0 else [()])
        out = torch.empty(sh["dim"], dtype=torch.float64, device=workspace.device)
        self._check(self.L.mbefci_tuple_hdiag(self.ptr, order, _p(t) if t.size else None,
                                              ctypes.c_void_p(workspace.data_ptr()), workspace.numel(),
                                              ctypes.c_void_p(out.data_ptr())))
        return out

    def class_stats(self) -> list:
        """Per-shape-class counters of the last call (list of dicts)."""
        n = ctypes.c_int32(0)
        self._check(self.L.mbefci_get_class_stats(self.ptr, ctypes.byref(n), None))
        arr = (_lib.ClassStats * max(1, n.value))()
        self._check(self.L.mbefci_get_class_stats(self.ptr, ctypes.byref(n), ctypes.cast(arr, ctypes.c_void_p)))
        return [{name: getattr(arr[i], name) for name, _ in _lib.ClassStats._fields_} for i in range(n.value)]

    def stats(self) -> dict:
        s = _lib.Stats()
        self._check(self.L.mbefci_get_stats(self.ptr, ctypes.byref(s)))
        return {name: getattr(s, name) for name, _ in _lib.Stats._fields_}


class ResultHandle:
    """Owns a library-side result (freed with the handle)."""

    def __init__(self, L, ptr):
        self.L, self.ptr = L, ptr

    def __del__(self):
        try:
            if self.ptr:
                self.L.mbefci_result_free(self.ptr)
                self.ptr = None
        except Exception:
            pass


def string_tables(n_active, nel):
    """(strings uint32 [nstr], links uint32 [nstr, nent]) of one shape (host)."""
    L = _lib.load()
    ns, ne = ctypes.c_int64(), ctypes.c_int32()
    rc = L.mbefci_string_tables(n_active, nel, ctypes.byref(ns), ctypes.byref(ne), None, None)
    if rc != 0:
        raise MBEFCIError(rc, "string_tables")
    s = np.zeros(ns.value, dtype=np.uint32)
    lk = np.zeros(ns.value * ne.value, dtype=np.uint32)
    L.mbefci_string_tables(n_active, nel, None, None, _p(s), _p(lk) if lk.size else None)
    return s, lk.reshape(ns.value, ne.value)


def workspace(nbytes: int, device=0):
    """Device workspace as a torch uint8 tensor."""
    import torch
    return torch.empty(int(nbytes), dtype=torch.uint8, device=f"cuda:{device}")
