"""ctypes binding of libsdc.so (include/sdc.h): argument marshalling only.

Every call forwards device pointers of torch tensors and the current HIP
stream to the C ABI; all arithmetic runs in the library's HIP kernels.  If the
library is not built this module raises instead of falling back to anything.
"""
from __future__ import annotations

import ctypes
import os
from ctypes import POINTER, byref, c_char_p, c_double, c_int, c_int32, c_int64, c_void_p

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libsdc.so")

SDC_FP64, SDC_MIXED = 0, 1
NODE_TYPES = {"lobatto": 0, "radau": 1}
MAX_NODES = 5
NSTATS = 21
ERRORS = {1: "SDC_ERR_ARG", 2: "SDC_ERR_HIP", 3: "SDC_ERR_NOMEM", 4: "SDC_ERR_NEWTON",
          5: "SDC_ERR_NONFINITE", 6: "SDC_ERR_UNSUPPORTED", 7: "SDC_ERR_COMPILE"}
EXPORTS = ("sdc_config_default", "sdc_init", "sdc_destroy", "sdc_last_error", "sdc_sizes",
           "sdc_advective_term", "sdc_source", "sdc_reaction_solve", "sdc_sweep", "sdc_step",
           "sdc_stats", "sdc_check", "sdc_stats_reset", "sdc_set_params", "sdc_compile_only",
           "sdc_generated_source", "sdc_aot_name", "sdc_profile_enable", "sdc_profile_read", "sdc_cost_model",
           "sdc_step_adjoint", "sdc_set_schedule", "sdc_get_schedule", "sdc_autotune",
           "sdc_reaction_solve_noalloc", "sdc_amr_create", "sdc_amr_destroy", "sdc_amr_sizes", "sdc_amr_handles",
           "sdc_amr_fill_patches", "sdc_amr_step")
KINDS = ("advect", "source", "solve", "transition_first", "transition_node0", "transition_later", "fill",
         "adjoint", "finish", "split", "order4")


class SDCError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{ERRORS.get(code, code)}: {msg}")
        self.code = code


class Network(ctypes.Structure):
    _fields_ = [("nspec", c_int32), ("nreact", c_int32), ("reactants", POINTER(c_int32)),
                ("stoich", POINTER(c_double)), ("lnA", POINTER(c_double)), ("b", POINTER(c_double)),
                ("E", POINTER(c_double)), ("q", POINTER(c_double))]


class Config(ctypes.Structure):
    _fields_ = [("dim", c_int32), ("n", c_int64 * 3), ("dx", c_double * 3), ("gamma", c_double),
                ("n_nodes", c_int32), ("n_iters", c_int32), ("precision", c_int32),
                ("advection", c_int32), ("slope", c_int32), ("alpha", c_double),
                ("newton_tol", c_double), ("newton_maxiter", c_int32),
                ("pivot_threshold", c_double), ("nbox", c_int32), ("box_n", POINTER(c_int64)),
                ("graph", c_int32), ("autotune", c_int32), ("node_type", c_int32),
                ("space_order", c_int32)]


class Patches(ctypes.Structure):
    _fields_ = [("npatch", c_int32), ("lo", POINTER(c_int64)), ("ext", POINTER(c_int64))]


class Nodes(ctypes.Structure):
    _fields_ = [("U", c_void_p * MAX_NODES), ("A", c_void_p * MAX_NODES),
                ("R", c_void_p * MAX_NODES), ("C", c_void_p * (MAX_NODES - 2))]


_lib = None


def lib():
    """The loaded libsdc.so; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is not built (python -m paper_1910_12578_amd.build)")
        # torch's HIP runtime (and hipRTC) must be the one libsdc.so binds to:
        # both carry the soname libamdhip64.so.7, and the first one loaded wins.
        import torch  # noqa: F401
        L = ctypes.CDLL(LIB_PATH)
        L.sdc_config_default.argtypes = [POINTER(Config)]
        L.sdc_init.argtypes = [POINTER(Config), POINTER(Network), POINTER(c_void_p)]
        L.sdc_destroy.argtypes = [c_void_p]
        L.sdc_last_error.argtypes = [c_void_p]
        L.sdc_last_error.restype = c_char_p
        L.sdc_sizes.argtypes = [c_void_p, POINTER(c_int64), POINTER(c_int32), POINTER(c_int32)]
        L.sdc_advective_term.argtypes = [c_void_p, c_void_p, c_void_p, c_void_p]
        L.sdc_source.argtypes = [c_void_p, c_void_p, c_void_p, c_void_p]
        L.sdc_reaction_solve.argtypes = [c_void_p, c_double, c_void_p, c_void_p, c_void_p, c_void_p,
                                         c_void_p, c_void_p]
        L.sdc_reaction_solve_noalloc.argtypes = [c_void_p, c_double, c_int64, c_void_p, c_void_p, c_void_p,
                                                 c_void_p, c_void_p, c_void_p]
        L.sdc_amr_create.argtypes = [POINTER(Config), POINTER(Network), POINTER(Patches), POINTER(c_void_p)]
        L.sdc_amr_destroy.argtypes = [c_void_p]
        L.sdc_amr_sizes.argtypes = [c_void_p, POINTER(c_int64), POINTER(c_int64)]
        L.sdc_amr_handles.argtypes = [c_void_p, POINTER(c_void_p), POINTER(c_void_p)]
        L.sdc_amr_fill_patches.argtypes = [c_void_p, c_void_p, c_void_p, c_void_p]
        L.sdc_amr_step.argtypes = [c_void_p, c_double, c_int32, c_void_p, c_void_p, c_void_p]
        L.sdc_sweep.argtypes = [c_void_p, c_double, c_int32, POINTER(Nodes), c_void_p]
        L.sdc_step.argtypes = [c_void_p, c_double, c_int32, c_void_p, POINTER(Nodes), c_void_p]
        L.sdc_stats.argtypes = [c_void_p, POINTER(c_int64)]
        L.sdc_check.argtypes = [c_void_p]
        L.sdc_stats_reset.argtypes = [c_void_p, c_void_p]
        L.sdc_set_params.argtypes = [c_void_p, POINTER(c_double), POINTER(c_double)]
        L.sdc_compile_only.argtypes = [POINTER(Config), POINTER(Network)]
        L.sdc_generated_source.argtypes = [POINTER(Config), POINTER(Network), c_char_p, c_int64]
        L.sdc_generated_source.restype = c_int64
        L.sdc_aot_name.argtypes = [POINTER(Config), POINTER(Network), c_char_p, c_int64]
        L.sdc_aot_name.restype = c_int64
        L.sdc_profile_enable.argtypes = [c_void_p, c_int32]
        L.sdc_profile_read.argtypes = [c_void_p, POINTER(c_double), POINTER(c_int64)]
        L.sdc_cost_model.argtypes = [c_void_p, POINTER(c_int64)]
        L.sdc_step_adjoint.argtypes = [c_void_p, c_double, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p]
        L.sdc_set_schedule.argtypes = [c_void_p, c_int32, c_int32, c_int32, c_int32]
        L.sdc_get_schedule.argtypes = [c_void_p, POINTER(c_int32), POINTER(c_int32), POINTER(c_int32),
                                       POINTER(c_int32)]
        L.sdc_autotune.argtypes = [c_void_p, c_double, c_void_p, POINTER(Nodes), c_void_p]
        for name in EXPORTS:
            getattr(L, name).restype = getattr(L, name).restype or c_int
        _lib = L
    return _lib


def _dptr(a):
    return a.ctypes.data_as(POINTER(c_double))


def make_network(net):
    """ctypes network struct plus the numpy arrays that must outlive it."""
    keep = dict(
        reactants=np.ascontiguousarray(net["reactants"], dtype=np.int32).reshape(-1, 2),
        stoich=np.ascontiguousarray(net["stoich"], dtype=np.float64),
        lnA=np.ascontiguousarray(net["lnA"], dtype=np.float64),
        b=np.ascontiguousarray(net["b"], dtype=np.float64),
        E=np.ascontiguousarray(net["E"], dtype=np.float64),
        q=np.ascontiguousarray(net["q"], dtype=np.float64),
    )
    n = Network(int(net["nspec"]), int(net["nreact"]),
                keep["reactants"].ctypes.data_as(POINTER(c_int32)), _dptr(keep["stoich"]),
                _dptr(keep["lnA"]), _dptr(keep["b"]), _dptr(keep["E"]), _dptr(keep["q"]))
    return n, keep


def make_config(cfg):
    """ctypes config struct; a box table, if any, is kept alive on the struct."""
    c = Config()
    lib().sdc_config_default(byref(c))
    c.dim = int(cfg["dim"])
    if cfg.get("box_n") is not None:
        boxes = np.ascontiguousarray(cfg["box_n"], dtype=np.int64).reshape(-1, 3)
        c.nbox = boxes.shape[0]
        c.box_n = boxes.ctypes.data_as(POINTER(c_int64))
        c._keep_boxes = boxes
    for d in range(3):
        c.n[d] = int(cfg["n"][d]) if d < len(cfg["n"]) else 1
        c.dx[d] = float(cfg["dx"][d]) if d < len(cfg["dx"]) else 1.0
    for key in ("gamma", "alpha", "newton_tol", "pivot_threshold"):
        if key in cfg:
            setattr(c, key, float(cfg[key]))
    if "node_type" in cfg:
        c.node_type = NODE_TYPES[cfg["node_type"]] if isinstance(cfg["node_type"], str) else int(cfg["node_type"])
    for key in ("n_nodes", "n_iters", "precision", "advection", "slope", "newton_maxiter", "graph", "autotune",
                "space_order"):
        if key in cfg:
            setattr(c, key, int(cfg[key]))
    return c


def config_from_workload(w, **over):
    """Config dict of an `sdc_inputs.workload` record (x-first extents)."""
    cfg = dict(dim=w["dim"], n=tuple(w["shape"] or ()), dx=tuple(w["dx"]), gamma=w["gamma"],
               n_nodes=w["n_nodes"], n_iters=w["n_iters"], precision=SDC_FP64, advection=1,
               slope=w["slope"], alpha=w["alpha"], newton_tol=w["newton_tol"],
               newton_maxiter=w["newton_maxiter"], node_type=w.get("node_type", "lobatto"),
               space_order=w.get("space_order", 2))
    if w.get("box_n") is not None:
        cfg["box_n"] = w["box_n"]
    cfg.update(over)
    return cfg


def _check(rc, handle=None):
    if rc != 0:
        msg = lib().sdc_last_error(handle)
        raise SDCError(rc, msg.decode() if msg else "")


def generated_source(cfg, net):
    c = make_config(cfg)
    n, _keep = make_network(net)
    need = lib().sdc_generated_source(byref(c), byref(n), None, 0)
    if need < 0:
        _check(-need)
    buf = ctypes.create_string_buffer(int(need))
    lib().sdc_generated_source(byref(c), byref(n), buf, need)
    return buf.value.decode()


def aot_name(cfg, net):
    """Path at which the runtime looks for the hipcc-built code object of
    `cfg` and `net` before compiling with hipRTC."""
    c = make_config(cfg)
    n, _keep = make_network(net)
    need = lib().sdc_aot_name(byref(c), byref(n), None, 0)
    if need < 0:
        _check(-need)
    buf = ctypes.create_string_buffer(int(need))
    lib().sdc_aot_name(byref(c), byref(n), buf, need)
    return buf.value.decode()


def compile_only(cfg, net):
    c = make_config(cfg)
    n, _keep = make_network(net)
    _check(lib().sdc_compile_only(byref(c), byref(n)))


class SDC:
    """One configured SDC solver on the current GPU (wraps an sdc_handle)."""

    def __init__(self, cfg: dict, net: dict):
        self.cfg = dict(cfg)
        self.net = net
        c = make_config(cfg)
        n, keep = make_network(net)
        h = c_void_p()
        _check(lib().sdc_init(byref(c), byref(n), byref(h)))
        self._h = h
        Z, nc, nx = c_int64(), c_int32(), c_int32()
        _check(lib().sdc_sizes(h, byref(Z), byref(nc), byref(nx)), h)
        self.zones, self.ncomp, self.nreact_vars = Z.value, nc.value, nx.value
        self.n_nodes = c.n_nodes
        self.nspec = int(net["nspec"])
        self.nreact = int(net["nreact"])

    # -- plumbing
    def close(self):
        if getattr(self, "_h", None):
            lib().sdc_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    @staticmethod
    def _stream(stream):
        import torch
        s = stream if stream is not None else torch.cuda.current_stream()
        return c_void_p(s.cuda_stream)

    def _ptr(self, t, ncomp, dtype=None):
        import torch
        dtype = dtype or torch.float64
        if not isinstance(t, torch.Tensor) or not t.is_cuda:
            raise TypeError("expected a CUDA (HIP) tensor")
        if t.dtype != dtype:
            raise TypeError(f"expected {dtype}, got {t.dtype}")
        if not t.is_contiguous():
            raise ValueError("tensor must be contiguous")
        if t.numel() != ncomp * self.zones:
            raise ValueError(f"expected {ncomp} x {self.zones} elements, got {tuple(t.shape)}")
        return c_void_p(t.data_ptr())

    def empty(self, ncomp, dtype=None):
        import torch
        return torch.empty((ncomp, self.zones), dtype=dtype or torch.float64, device="cuda")

    # -- C ABI calls
    def advective_term(self, U, A=None, stream=None):
        A = self.empty(self.ncomp) if A is None else A
        _check(lib().sdc_advective_term(self._h, self._ptr(U, self.ncomp), self._ptr(A, self.ncomp),
                                        self._stream(stream)), self._h)
        return A

    def source(self, U, R=None, stream=None):
        R = self.empty(self.nreact_vars) if R is None else R
        _check(lib().sdc_source(self._h, self._ptr(U, self.ncomp), self._ptr(R, self.nreact_vars),
                                self._stream(stream)), self._h)
        return R

    def reaction_solve(self, dtm, rho, b, x, R=None, iters=None, stream=None):
        import torch
        R = self.empty(self.nreact_vars) if R is None else R
        iters = torch.empty(self.zones, dtype=torch.int32, device="cuda") if iters is None else iters
        _check(lib().sdc_reaction_solve(self._h, float(dtm), self._ptr(rho, 1), self._ptr(b, self.nreact_vars),
                                        self._ptr(x, self.nreact_vars), self._ptr(R, self.nreact_vars),
                                        self._ptr(iters, 1, torch.int32), self._stream(stream)), self._h)
        return x, R, iters

    def reaction_solve_noalloc(self, dtm, rho, b, x, R, iters, stream=None):
        """sdc_reaction_solve_noalloc on the zones of `rho` ([nz]); b, x, R:
        [n_r][nz], iters: int32 [nz], all preallocated by the caller."""
        import torch
        nz = rho.numel()
        for t, nc, dt in ((rho, 1, torch.float64), (b, self.nreact_vars, torch.float64),
                          (x, self.nreact_vars, torch.float64), (R, self.nreact_vars, torch.float64),
                          (iters, 1, torch.int32)):
            if not isinstance(t, torch.Tensor) or not t.is_cuda or t.dtype != dt or not t.is_contiguous():
                raise TypeError(f"expected a contiguous CUDA tensor of {dt}")
            if t.numel() != nc * nz:
                raise ValueError(f"expected {nc} x {nz} elements, got {tuple(t.shape)}")
        _check(lib().sdc_reaction_solve_noalloc(self._h, float(dtm), nz, c_void_p(rho.data_ptr()),
                                                c_void_p(b.data_ptr()), c_void_p(x.data_ptr()),
                                                c_void_p(R.data_ptr()), c_void_p(iters.data_ptr()),
                                                self._stream(stream)), self._h)
        return x, R, iters

    def alloc_nodes(self):
        M = self.n_nodes - 1
        return dict(U=[self.empty(self.ncomp) for _ in range(M + 1)],
                    A=[self.empty(self.ncomp) for _ in range(M + 1)],
                    R=[self.empty(self.nreact_vars) for _ in range(M + 1)],
                    C=[self.empty(self.ncomp) for _ in range(max(M - 1, 0))])

    def _nodes(self, nodes):
        n = Nodes()
        for key, nc, cnt in (("U", self.ncomp, MAX_NODES), ("A", self.ncomp, MAX_NODES),
                             ("R", self.nreact_vars, MAX_NODES), ("C", self.ncomp, MAX_NODES - 2)):
            arr = getattr(n, key)
            for j, t in enumerate(nodes.get(key, [])):
                if t is not None:
                    arr[j] = self._ptr(t, nc).value
        return n

    def sweep(self, dt, k, nodes, stream=None):
        n = self._nodes(nodes)
        _check(lib().sdc_sweep(self._h, float(dt), int(k), byref(n), self._stream(stream)), self._h)

    def step(self, dt, nsteps, U, work=None, stream=None):
        work = self.alloc_nodes() if work is None else work
        n = self._nodes(work)
        _check(lib().sdc_step(self._h, float(dt), int(nsteps), self._ptr(U, self.ncomp), byref(n),
                              self._stream(stream)), self._h)
        return U

    def step_adjoint(self, dt, U_n, Ubar_np1, Ubar_n=None, thetabar=None, stream=None):
        """One step backward: Ubar_n = (dU^{n+1}/dU^n)^T Ubar_np1; thetabar += parameter adjoints."""
        import torch
        Ubar_n = self.empty(self.ncomp) if Ubar_n is None else Ubar_n
        if thetabar is None:
            thetabar = torch.zeros(2 * max(self.nreact, 1), dtype=torch.float64, device="cuda")
        if thetabar.numel() < 2 * self.nreact or not thetabar.is_cuda or thetabar.dtype != torch.float64:
            raise ValueError("thetabar must be a float64 CUDA tensor with 2 * nreact entries")
        _check(lib().sdc_step_adjoint(self._h, float(dt), self._ptr(U_n, self.ncomp), self._ptr(Ubar_np1, self.ncomp),
                                      self._ptr(Ubar_n, self.ncomp), c_void_p(thetabar.data_ptr()),
                                      self._stream(stream)), self._h)
        return Ubar_n, thetabar

    def generated_source(self):
        """The device source this handle compiled (generated network code + kernels)."""
        return generated_source(self.cfg, self.net)

    def set_schedule(self, occ2, cap, split=0, zchunk=0):
        _check(lib().sdc_set_schedule(self._h, int(occ2), int(cap), int(split), int(zchunk)), self._h)

    def schedule(self):
        """(occ2, cap, split, zchunk)"""
        o, c, sp, zt = c_int32(), c_int32(), c_int32(), c_int32()
        _check(lib().sdc_get_schedule(self._h, byref(o), byref(c), byref(sp), byref(zt)), self._h)
        return o.value, c.value, sp.value, zt.value

    def autotune(self, dt, U, work=None, stream=None):
        work = self.alloc_nodes() if work is None else work
        n = self._nodes(work)
        _check(lib().sdc_autotune(self._h, float(dt), self._ptr(U, self.ncomp), byref(n), self._stream(stream)),
               self._h)
        return self.schedule()

    def stats(self):
        out = (c_int64 * NSTATS)()
        _check(lib().sdc_stats(self._h, out), self._h)
        v = list(out)
        return dict(hist=v[0:16], failed=v[16], iters=v[17], nonfinite=v[18], solves=v[19], fallbacks=v[20])

    def check(self):
        """Device-side outcome since the last stats reset: 0 (all solves converged
        and finite), 4 (SDC_ERR_NEWTON) or 5 (SDC_ERR_NONFINITE), with the
        library's description of the counts."""
        rc = lib().sdc_check(self._h)
        if rc not in (0, 4, 5):
            _check(rc, self._h)
        msg = lib().sdc_last_error(self._h)
        return rc, (msg.decode() if msg and rc else "")

    def stats_reset(self, stream=None):
        _check(lib().sdc_stats_reset(self._h, self._stream(stream)), self._h)

    def profile(self, enable=True):
        _check(lib().sdc_profile_enable(self._h, int(bool(enable))), self._h)

    def profile_read(self):
        """{kind: (milliseconds, launches)} since the last read."""
        ms = (c_double * len(KINDS))()
        n = (c_int64 * len(KINDS))()
        _check(lib().sdc_profile_read(self._h, ms, n), self._h)
        return {k: (ms[i], n[i]) for i, k in enumerate(KINDS)}

    def cost_model(self):
        out = (c_int64 * 7)()
        _check(lib().sdc_cost_model(self._h, out), self._h)
        keys = ("source", "residual_matrix", "lu", "solve", "exps", "nnz_jac", "nnz_lu")
        return dict(zip(keys, list(out)))

    def set_params(self, lnA, E):
        lnA = np.ascontiguousarray(lnA, dtype=np.float64)
        E = np.ascontiguousarray(E, dtype=np.float64)
        if lnA.size != self.nreact or E.size != self.nreact:
            raise ValueError("expected one lnA and one E per reaction")
        _check(lib().sdc_set_params(self._h, _dptr(lnA), _dptr(E)), self._h)


class AMR:
    """Two-level hierarchy (refined patches with subcycling) on the current
    GPU: wraps an sdc_amr.  `patches` is a list of (lo, ext) in coarse zones,
    x first."""

    def __init__(self, cfg: dict, net: dict, patches):
        c = make_config(cfg)
        n, keep = make_network(net)
        lo = np.zeros((len(patches), 3), dtype=np.int64)
        ext = np.ones((len(patches), 3), dtype=np.int64)
        for i, (pl, pe) in enumerate(patches):
            lo[i, :len(pl)] = pl
            ext[i, :len(pe)] = pe
        pt = Patches(len(patches), lo.ctypes.data_as(POINTER(c_int64)), ext.ctypes.data_as(POINTER(c_int64)))
        a = c_void_p()
        _check(lib().sdc_amr_create(byref(c), byref(n), byref(pt), byref(a)))
        self._a = a
        zc, zf = c_int64(), c_int64()
        lib().sdc_amr_sizes(a, byref(zc), byref(zf))
        self.zc, self.zf = zc.value, zf.value
        hc, hf = c_void_p(), c_void_p()
        lib().sdc_amr_handles(a, byref(hc), byref(hf))
        self._hc, self._hf = hc, hf
        self.ncomp = 2 + int(cfg["dim"]) + int(net["nspec"])

    def _arr(self, t, zones):
        import torch
        if not isinstance(t, torch.Tensor) or not t.is_cuda or t.dtype != torch.float64 or not t.is_contiguous():
            raise TypeError("expected a contiguous float64 CUDA tensor")
        if t.numel() != self.ncomp * zones:
            raise ValueError(f"expected {self.ncomp} x {zones} elements, got {tuple(t.shape)}")
        return c_void_p(t.data_ptr())

    def fill_patches(self, Uc, Uf, stream=None):
        _check(lib().sdc_amr_fill_patches(self._a, self._arr(Uc, self.zc), self._arr(Uf, self.zf),
                                          SDC._stream(stream)), self._hc)

    def step(self, dt, nsteps, Uc, Uf, stream=None):
        _check(lib().sdc_amr_step(self._a, float(dt), int(nsteps), self._arr(Uc, self.zc), self._arr(Uf, self.zf),
                                  SDC._stream(stream)), self._hc)

    def set_schedule(self, occ2=0, cap=0, split=0, zchunk=0):
        """sdc_set_schedule on the coarse level; a step passes its Newton
        schedule (occ2, cap) on to the patches."""
        _check(lib().sdc_set_schedule(self._hc, int(occ2), int(cap), int(split), int(zchunk)), self._hc)

    def stats(self):
        out = []
        for h in (self._hc, self._hf):
            v = (c_int64 * NSTATS)()
            _check(lib().sdc_stats(h, v), h)
            v = list(v)
            out.append(dict(hist=v[0:16], failed=v[16], iters=v[17], nonfinite=v[18], solves=v[19]))
        return out

    def close(self):
        if getattr(self, "_a", None):
            lib().sdc_amr_destroy(self._a)
            self._a = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
