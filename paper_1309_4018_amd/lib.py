"""ctypes binding of libpbtc (argument marshalling only).

Every computation happens in the HIP library; this module only converts
arrays, owns the device workspace (a torch uint8 CUDA tensor, so that torch's
caching allocator supplies the memory) and passes the current HIP stream.
Loading fails loudly when the library has not been built.
"""

from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libpbtc.so")

OK, EINVAL, EMESH, ECHARGE, EWORKSPACE, EDEVICE, ENOCONV, EHOST = 0, -1, -2, -3, -4, -5, -6, -7
FP64, FP32_REFINED, FP32 = 0, 1, 2
OP_TREECODE, OP_DIRECT = 0, 1
PREC_NONE, PREC_BLOCK_DIAG = 0, 1

_ERRNAMES = {EINVAL: "EINVAL", EMESH: "EMESH", ECHARGE: "ECHARGE", EWORKSPACE: "EWORKSPACE",
             EDEVICE: "EDEVICE", ENOCONV: "ENOCONV", EHOST: "EHOST"}


class TreeSizes(C.Structure):
    _fields_ = [("n_cells", C.c_int64), ("n_gauss_points", C.c_int64), ("n_targets", C.c_int64),
                ("n_groups", C.c_int64), ("n_items", C.c_int64), ("n_near", C.c_int64),
                ("n_far", C.c_int64), ("n_surfaces", C.c_int), ("ncrit", C.c_int)]


class Params(C.Structure):
    _fields_ = [
        ("K", C.c_int), ("K_fine", C.c_int), ("N_k", C.c_int), ("thres", C.c_double),
        ("theta", C.c_double), ("P", C.c_int), ("ncrit", C.c_int), ("direct_below", C.c_int),
        ("tol", C.c_double), ("restart", C.c_int), ("max_iter", C.c_int),
        ("precision", C.c_int), ("op", C.c_int), ("inner_tol", C.c_double),
        ("max_refine", C.c_int), ("validate_charges", C.c_int), ("profile", C.c_int),
        ("precond", C.c_int), ("unit_sources", C.c_int), ("unit_cells", C.c_int),
        ("op_graph", C.c_int),
    ]


class Result(C.Structure):
    _fields_ = [
        ("energy_kJmol", C.c_double), ("n_iter", C.c_int), ("converged", C.c_int),
        ("final_rel_res", C.c_double), ("n_matvec_fp32", C.c_int), ("n_matvec_fp64", C.c_int),
        ("n_refine", C.c_int), ("t_setup_s", C.c_double), ("t_solve_s", C.c_double),
        ("t_energy_s", C.c_double), ("n_p2p_pairs", C.c_double), ("n_m2p_evals", C.c_double),
        ("n_dense_equiv", C.c_double), ("n_near_entries", C.c_double),
        ("workspace_needed", C.c_size_t),
        ("t_p2p_s", C.c_double), ("t_m2p_s", C.c_double),
        ("n_p2p_launch", C.c_int), ("n_m2p_launch", C.c_int),
        ("p2p_flop", C.c_double), ("m2p_flop", C.c_double),
        ("t_m2p_yuk_s", C.c_double), ("n_m2p_yuk_launch", C.c_int),
        ("m2p_yuk_flop", C.c_double),
        ("t_setup_phase_s", C.c_double * 6),
        ("op_kernels", C.c_int), ("op_graph_launches", C.c_int),
        ("t_kernel_s", C.c_double * 7), ("n_kernel_launch", C.c_int * 7),
        ("kernel_flop", C.c_double * 7),
        ("tile_sources", C.c_int), ("tile_cells", C.c_int),
    ]

    def as_dict(self):
        out = {}
        for k, _ in self._fields_:
            v = getattr(self, k)
            out[k] = list(v) if isinstance(v, C.Array) else v
        return out


_EXPORTS = {
    "pbtc_version": (C.c_int, [C.POINTER(C.c_int), C.POINTER(C.c_int)]),
    "pbtc_problem_create": (C.c_int, [C.POINTER(C.c_void_p)]),
    "pbtc_problem_destroy": (None, [C.c_void_p]),
    "pbtc_add_region": (C.c_int, [C.c_void_p, C.c_double, C.c_double, C.POINTER(C.c_int)]),
    "pbtc_add_surface": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int64, C.c_void_p, C.c_int64,
                                   C.c_int, C.c_int, C.POINTER(C.c_int)]),
    "pbtc_set_charges": (C.c_int, [C.c_void_p, C.c_int, C.c_void_p, C.c_void_p, C.c_int64]),
    "pbtc_params_default": (C.c_int, [C.POINTER(Params)]),
    "pbtc_validate": (C.c_int, [C.c_void_p, C.POINTER(Params)]),
    "pbtc_plan": (C.c_int, [C.c_void_p, C.POINTER(Params), C.POINTER(C.c_void_p),
                            C.POINTER(C.c_size_t)]),
    "pbtc_plan_destroy": (None, [C.c_void_p]),
    "pbtc_plan_sizes": (C.c_int, [C.c_void_p, C.POINTER(C.c_int64), C.POINTER(C.c_int64),
                                  C.POINTER(C.c_int), C.POINTER(C.c_int)]),
    "pbtc_setup": (C.c_int, [C.c_void_p, C.c_void_p, C.c_size_t, C.c_void_p, C.POINTER(Result)]),
    "pbtc_solve": (C.c_int, [C.c_void_p, C.c_void_p, C.c_size_t, C.c_void_p, C.c_int,
                             C.POINTER(Result)]),
    "pbtc_solve_batch": (C.c_int, [C.POINTER(C.c_void_p), C.c_int, C.c_void_p, C.c_size_t,
                                   C.c_void_p, C.POINTER(Result)]),
    "pbtc_get_surface": (C.c_int, [C.c_void_p, C.c_int, C.c_void_p, C.c_void_p]),
    "pbtc_get_phi_reac": (C.c_int, [C.c_void_p, C.c_void_p]),
    "pbtc_get_history": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int, C.POINTER(C.c_int)]),
    "pbtc_matvec": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_int]),
    "pbtc_matvec_transpose": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
                                        C.c_void_p, C.c_int]),
    "pbtc_precond_apply": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
                                     C.c_void_p, C.c_int]),
    "pbtc_coulomb_energy": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
                                      C.c_void_p]),
    "pbtc_coulomb_energy_noalloc": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
                                              C.c_void_p]),
    "pbtc_rhs": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]),
    "pbtc_backward": (C.c_int, [C.c_void_p, C.c_void_p, C.c_size_t, C.c_void_p, C.c_double,
                                C.c_void_p, C.c_void_p, C.c_void_p, C.POINTER(Result)]),
    "pbtc_get_tree": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.POINTER(TreeSizes)]
                      + [C.c_void_p] * 10),
    "pbtc_get_systems": (C.c_int, [C.c_void_p, C.POINTER(C.c_int), C.c_void_p, C.c_void_p,
                                   C.c_void_p]),
    "pbtc_set_charge_values": (C.c_int, [C.c_void_p, C.c_void_p]),
    "pbtc_triangle_rule": (C.c_int, [C.c_int, C.c_void_p, C.c_void_p]),
    "pbtc_gauss_legendre": (C.c_int, [C.c_int, C.c_void_p, C.c_void_p]),
    "pbtc_last_error": (C.c_char_p, [C.c_void_p]),
}

_lib = None


class PbtcError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{_ERRNAMES.get(code, code)}: {msg}")
        self.code = code


def load(path: str | None = None):
    """Loads libpbtc.so (built in place by ``paper_1309_4018_amd.build``)."""
    global _lib
    if _lib is not None and path is None:
        return _lib
    p = path or LIB_PATH
    # torch ships its own HIP runtime under the same soname as the system
    # one; torch is loaded first so that the library binds to that runtime
    # and both share devices, streams and memory.
    import torch  # noqa: F401
    if not os.path.exists(p):
        raise RuntimeError(
            f"{p} is missing: build it with `python -m paper_1309_4018_amd.build` "
            "(there is no fallback implementation)")
    lib = C.CDLL(p)
    for name, (res, args) in _EXPORTS.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    if path is None:
        _lib = lib
    return lib


def exported_names():
    return list(_EXPORTS)


def _ptr(a):
    return C.c_void_p(a.ctypes.data) if a is not None else None


def check(code, plan=None):
    if code == OK:
        return
    lib = load()
    msg = lib.pbtc_last_error(plan)
    raise PbtcError(code, msg.decode() if msg else "")


def default_params(**kw):
    p = Params()
    check(load().pbtc_params_default(C.byref(p)))
    prec = kw.pop("precision", None)
    if isinstance(prec, str):
        kw["precision"] = {"fp64": FP64, "fp32_refined": FP32_REFINED, "fp32": FP32}[prec]
    elif prec is not None:
        kw["precision"] = prec
    op = kw.pop("op", None)
    if isinstance(op, str):
        kw["op"] = {"treecode": OP_TREECODE, "direct": OP_DIRECT}[op]
    elif op is not None:
        kw["op"] = op
    pc = kw.pop("precond", None)
    if isinstance(pc, str):
        kw["precond"] = {"none": PREC_NONE, "block_diag": PREC_BLOCK_DIAG}[pc]
    elif pc is not None:
        kw["precond"] = pc
    for k, v in kw.items():
        if not hasattr(p, k):
            raise KeyError(k)
        setattr(p, k, v)
    return p


class Problem:
    """Host-side problem description (regions, surfaces, charges)."""

    def __init__(self):
        self.lib = load()
        h = C.c_void_p()
        check(self.lib.pbtc_problem_create(C.byref(h)))
        self.h = h
        self.surface_sizes = []

    def __del__(self):
        if getattr(self, "h", None):
            self.lib.pbtc_problem_destroy(self.h)
            self.h = None

    def add_region(self, eps, kappa):
        rid = C.c_int()
        check(self.lib.pbtc_add_region(self.h, float(eps), float(kappa), C.byref(rid)))
        return rid.value

    def add_surface(self, verts, tris, inner, outer):
        v = np.ascontiguousarray(verts, dtype=np.float64).reshape(-1, 3)
        t = np.ascontiguousarray(tris, dtype=np.int32).reshape(-1, 3)
        sid = C.c_int()
        check(self.lib.pbtc_add_surface(self.h, _ptr(v), len(v), _ptr(t), len(t), int(inner),
                                        int(outer), C.byref(sid)))
        self.surface_sizes.append(len(t))
        return sid.value

    def set_charges(self, region, xyz, q):
        x = np.ascontiguousarray(xyz, dtype=np.float64).reshape(-1, 3)
        qq = np.ascontiguousarray(q, dtype=np.float64).reshape(-1)
        check(self.lib.pbtc_set_charges(self.h, int(region), _ptr(x), _ptr(qq), len(qq)))

    def validate(self, params=None):
        params = params or default_params()
        check(self.lib.pbtc_validate(self.h, C.byref(params)))

    @classmethod
    def from_synth(cls, prob):
        """From a ``synth.Problem``-like object (regions, surfaces, charges)."""
        p = cls()
        for r in prob.regions:
            p.add_region(r.eps, r.kappa)
        for s in prob.surfaces:
            p.add_surface(s.verts, s.tris, s.inner, s.outer)
        for r, (x, q) in prob.charges.items():
            p.set_charges(r, x, q)
        return p


def _stream_handle(torch, device):
    return C.c_void_p(torch.cuda.current_stream(device).cuda_stream)


class Plan:
    """A solver plan bound to one device workspace (torch uint8 tensor)."""

    def __init__(self, problem: Problem, params=None, device="cuda:0"):
        import torch

        self.torch = torch
        self.lib = load()
        self.problem = problem
        self.params = params or default_params()
        self.device = torch.device(device)
        h = C.c_void_p()
        nbytes = C.c_size_t()
        check(self.lib.pbtc_plan(problem.h, C.byref(self.params), C.byref(h), C.byref(nbytes)))
        self.h = h
        self.ws = None
        self._alloc(nbytes.value)
        n_unk, n_q, n_s, n_r = C.c_int64(), C.c_int64(), C.c_int(), C.c_int()
        check(self.lib.pbtc_plan_sizes(self.h, C.byref(n_unk), C.byref(n_q), C.byref(n_s),
                                       C.byref(n_r)), self.h)
        self.n_unknowns, self.n_charges = n_unk.value, n_q.value
        self.n_surfaces, self.n_regions = n_s.value, n_r.value
        self.problem_sizes = list(getattr(problem, "surface_sizes", []))
        self.last = Result()
        self.solve_count = 0  # completed solves (the autograd wrapper checks it)

    def __del__(self):
        if getattr(self, "h", None):
            self.lib.pbtc_plan_destroy(self.h)
            self.h = None

    def _alloc(self, nbytes):
        self.ws = self.torch.empty(int(nbytes), dtype=self.torch.uint8, device=self.device)

    @property
    def stream(self):
        return _stream_handle(self.torch, self.device)

    def _ws(self):
        return C.c_void_p(self.ws.data_ptr()), self.ws.numel()

    def _call_growing(self, fn):
        for _ in range(4):
            res = Result()
            ptr, n = self._ws()
            code = fn(ptr, n, res)
            if code == EWORKSPACE and res.workspace_needed > n:
                self._alloc(res.workspace_needed)
                continue
            self.last = res
            return code, res
        return code, res

    def setup(self):
        code, res = self._call_growing(
            lambda p, n, r: self.lib.pbtc_setup(self.h, p, n, self.stream, C.byref(r)))
        check(code, self.h)
        return res.as_dict()

    def solve(self, force_setup=False, allow_noconv=False):
        code, res = self._call_growing(
            lambda p, n, r: self.lib.pbtc_solve(self.h, p, n, self.stream, int(force_setup),
                                                C.byref(r)))
        if code in (OK, ENOCONV):
            self.solve_count += 1
        if not (allow_noconv and code == ENOCONV):
            check(code, self.h)
        return res.as_dict()

    def surface(self, sid):
        n = self._surface_size(sid)
        phi = np.empty(n)
        dphi = np.empty(n)
        check(self.lib.pbtc_get_surface(self.h, sid, _ptr(phi), _ptr(dphi)))
        return phi, dphi

    def _surface_size(self, sid):
        return self.problem_sizes[sid]

    def solution(self):
        """Unknown vector [phi_s, psi_s] per surface (host copy)."""
        out = []
        for sid in range(self.n_surfaces):
            out.extend(self.surface(sid))
        return np.concatenate(out)

    def phi_reac(self):
        out = np.empty(self.n_charges)
        check(self.lib.pbtc_get_phi_reac(self.h, _ptr(out)))
        return out

    def history(self):
        n = C.c_int()
        check(self.lib.pbtc_get_history(self.h, None, 0, C.byref(n)))
        out = np.empty(max(n.value, 1))
        check(self.lib.pbtc_get_history(self.h, _ptr(out), len(out), C.byref(n)))
        return out[:n.value]

    def matvec(self, x, precision=FP64, transpose=False):
        """A x (or A^T x) for a host or device vector; returns a torch tensor."""
        torch = self.torch
        xd = torch.as_tensor(np.asarray(x, dtype=np.float64) if not torch.is_tensor(x) else x,
                             dtype=torch.float64).to(self.device).contiguous()
        if xd.numel() != self.n_unknowns:
            raise ValueError("x has the wrong length")
        yd = torch.empty_like(xd)
        fn = self.lib.pbtc_matvec_transpose if transpose else self.lib.pbtc_matvec
        for _ in range(3):
            code = fn(self.h, C.c_void_p(self.ws.data_ptr()), self.stream,
                      C.c_void_p(xd.data_ptr()), C.c_void_p(yd.data_ptr()), int(precision))
            if code == EWORKSPACE and transpose:
                # the transposed operator needs more room: set up again at the
                # grown layout (the workspace grows on demand)
                self.setup()
                continue
            break
        check(code, self.h)
        return yd

    def precond_apply(self, x, transpose=False):
        """M^-1 x (or M^-T x) of the block-diagonal preconditioner."""
        torch = self.torch
        xd = torch.as_tensor(np.asarray(x, dtype=np.float64) if not torch.is_tensor(x) else x,
                             dtype=torch.float64).to(self.device).contiguous()
        if xd.numel() != self.n_unknowns:
            raise ValueError("x has the wrong length")
        yd = torch.empty_like(xd)
        check(self.lib.pbtc_precond_apply(self.h, C.c_void_p(self.ws.data_ptr()), self.stream,
                                          C.c_void_p(xd.data_ptr()), C.c_void_p(yd.data_ptr()),
                                          int(bool(transpose))), self.h)
        return yd

    def coulomb_energy(self):
        """(total, per system) Coulomb energy of the charges, kJ/mol."""
        n = C.c_int()
        check(self.lib.pbtc_get_systems(self.h, C.byref(n), None, None, None), self.h)
        per = np.empty(max(n.value, 1))
        tot = C.c_double()

        def call():
            return self.lib.pbtc_coulomb_energy(self.h, C.c_void_p(self.ws.data_ptr()),
                                                self.stream, C.byref(tot), _ptr(per))

        code = call()
        if code == EINVAL:  # not set up on this workspace yet
            self.setup()
            code = call()
        check(code, self.h)
        return tot.value, per[:n.value]

    def tree(self):
        """Octrees and forward interaction lists of the set-up (host copies)."""
        sz = TreeSizes()
        ws = C.c_void_p(self.ws.data_ptr())
        nulls = [None] * 10
        check(self.lib.pbtc_get_tree(self.h, ws, self.stream, C.byref(sz), *nulls), self.h)
        out = {
            "cells": np.empty((sz.n_cells, 9)),
            "gauss_points": np.empty((sz.n_gauss_points, 3)),
            "surface_gp": np.empty((sz.n_surfaces, 2), dtype=np.int64),
            "targets": np.empty((sz.n_targets, 3)),
            "groups": np.empty((sz.n_groups, 6)),
            "items": np.empty((sz.n_items, 4), dtype=np.int64),
            "near_ptr": np.empty(sz.n_items + 1, dtype=np.int64),
            "near": np.empty(max(sz.n_near, 1), dtype=np.int32),
            "far_ptr": np.empty(sz.n_items + 1, dtype=np.int64),
            "far": np.empty(max(sz.n_far, 1), dtype=np.int32),
        }
        keys = ["cells", "gauss_points", "surface_gp", "targets", "groups", "items", "near_ptr",
                "near", "far_ptr", "far"]
        check(self.lib.pbtc_get_tree(self.h, ws, self.stream, C.byref(sz),
                                     *[_ptr(out[k]) for k in keys]), self.h)
        out["ncrit"] = sz.ncrit
        return out

    def rhs(self):
        torch = self.torch
        b = torch.empty(self.n_unknowns, dtype=torch.float64, device=self.device)
        check(self.lib.pbtc_rhs(self.h, C.c_void_p(self.ws.data_ptr()), self.stream,
                                C.c_void_p(b.data_ptr())), self.h)
        return b

    def set_charge_values(self, q):
        qq = np.ascontiguousarray(q, dtype=np.float64).reshape(-1)
        if len(qq) != self.n_charges:
            raise ValueError("wrong number of charges")
        check(self.lib.pbtc_set_charge_values(self.h, _ptr(qq)), self.h)

    def backward(self, gE=1.0):
        """dE/dq (per charge), dE/dkappa and dE/deps (per region), times gE.

        The first call builds the transposed operator on the workspace; if
        the workspace must grow for it, the forward solve is repeated."""
        dq = np.empty(self.n_charges)
        dk = np.empty(self.n_regions)
        de = np.empty(self.n_regions)
        for _ in range(3):
            res = Result()
            code = self.lib.pbtc_backward(self.h, C.c_void_p(self.ws.data_ptr()), self.ws.numel(),
                                          self.stream, float(gE), _ptr(dq), _ptr(dk), _ptr(de),
                                          C.byref(res))
            if code == EWORKSPACE and res.workspace_needed > self.ws.numel():
                # the transposed operator needs more room: the forward solve of
                # the same charges (pbtc_backward accepts no others) is redone
                # on the larger workspace
                self._alloc(res.workspace_needed)
                self.solve()
                continue
            break
        check(code, self.h)
        self.last = res
        return dq, dk, de


def plan_for(prob, device="cuda:0", **params):
    """Problem + plan from a ``synth.Problem``; keeps the surface sizes."""
    p = Problem.from_synth(prob)
    return Plan(p, default_params(**params), device)


def batch_problem(problems):
    """One problem holding several independent molecules (``synth`` problems);
    the library solves each as its own system with shared kernel launches."""
    p = Problem()
    nreg = 0
    for prob in problems:
        for r in prob.regions:
            p.add_region(r.eps, r.kappa)
        for s in prob.surfaces:
            p.add_surface(s.verts, s.tris, nreg + s.inner, nreg + s.outer)
        for r, (x, q) in prob.charges.items():
            p.set_charges(nreg + r, x, q)
        nreg += len(prob.regions)
    return p


def systems(plan):
    """Per independent system: energy, explicit relative residual, first unknown."""
    n = C.c_int()
    check(plan.lib.pbtc_get_systems(plan.h, C.byref(n), None, None, None), plan.h)
    e = np.empty(n.value)
    r = np.empty(n.value)
    u = np.empty(n.value, dtype=np.int64)
    check(plan.lib.pbtc_get_systems(plan.h, C.byref(n), _ptr(e), _ptr(r), _ptr(u)), plan.h)
    return e, r, u


class Batch:
    """Several plans solved together by ``pbtc_solve_batch`` on one workspace
    (every kernel launch shared, every system with its own Krylov space)."""

    def __init__(self, plans):
        import torch

        self.torch = torch
        self.plans = list(plans)
        if not self.plans:
            raise ValueError("empty batch")
        self.lib = load()
        self.device = self.plans[0].device
        self._arr = (C.c_void_p * len(self.plans))(*[p.h for p in self.plans])
        self.ws = torch.empty(0, dtype=torch.uint8, device=self.device)

    def solve(self, allow_noconv=False):
        """Results (one dict per plan); the workspace grows on demand."""
        n = len(self.plans)
        for _ in range(4):
            res = (Result * n)()
            code = self.lib.pbtc_solve_batch(
                self._arr, n, C.c_void_p(self.ws.data_ptr() if self.ws.numel() else 0),
                self.ws.numel(), _stream_handle(self.torch, self.device), res)
            if code == EWORKSPACE and res[0].workspace_needed > self.ws.numel():
                self.ws = self.torch.empty(int(res[0].workspace_needed), dtype=self.torch.uint8,
                                           device=self.device)
                continue
            break
        if not (allow_noconv and code == ENOCONV):
            check(code, self.plans[0].h)
        for p, r in zip(self.plans, res):
            p.last = r
        return [r.as_dict() for r in res]


def triangle_rule(k):
    b = np.empty((k, 3))
    w = np.empty(k)
    check(load().pbtc_triangle_rule(k, _ptr(b), _ptr(w)))
    return b, w


def gauss_legendre(n):
    x = np.empty(n)
    w = np.empty(n)
    check(load().pbtc_gauss_legendre(n, _ptr(x), _ptr(w)))
    return x, w
