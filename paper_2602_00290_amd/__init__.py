"""Python binding of libtt_transport.so (ctypes; argument marshalling only).

Every step of the transport + rounding path runs in the library's HIP kernels;
this module converts a problem description into the C struct, allocates the
device workspace with PyTorch, and forwards calls.  There is no CPU fallback:
importing fails loudly when the shared library is missing.

Names follow the C ABI in include/tt_transport.h.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libtt_transport.so")

TT_OK, TT_ERR_INVALID_ARG, TT_ERR_OOM, TT_ERR_NUMERIC, TT_ERR_HIP, TT_ERR_STATE = 0, -1, -2, -3, -4, -5
TT_PREC_FP64, TT_PREC_FP32, TT_PREC_BF16X = 0, 1, 2
TT_ROUND_QR, TT_ROUND_GRAM, TT_ROUND_AUTO, TT_ROUND_RAND = 0, 1, 2, 3
TT_BC_VACUUM, TT_BC_INFLOW_PLANCK, TT_BC_PERIODIC, TT_BC_INFLOW_VALUES = 0, 1, 2, 3
TT_FLUX_UPWIND, TT_FLUX_RUSANOV, TT_FLUX_HLL = 0, 1, 2

KERNEL_CLASSES = ("prep", "project", "factor", "tree", "svd", "output", "diag", "couple", "angle", "stencil")

_dp = ctypes.POINTER(ctypes.c_double)


class TTProblem(ctypes.Structure):
    _fields_ = [
        ("dim", ctypes.c_int),
        ("n_cells", ctypes.c_int * 3),
        ("extent", ctypes.c_double * 3),
        ("n_groups", ctypes.c_int),
        ("group_edges", _dp),
        ("kappa0", _dp),
        ("kappa_group_scale", _dp),
        ("T_cell", _dp),
        ("n_theta", ctypes.c_int),
        ("n_phi", ctypes.c_int),
        ("mu", _dp),
        ("w_theta", _dp),
        ("phi", _dp),
        ("w_phi", _dp),
        ("bc", ctypes.c_int * 6),
        ("bc_T", ctypes.c_double * 6),
        ("bc_values", _dp),
        ("c", ctypes.c_double),
        ("cfl", ctypes.c_double),
        ("tol", ctypes.c_double),
        ("rank_cap", ctypes.c_int),
        ("precision", ctypes.c_int),
        ("round_method", ctypes.c_int),
        ("paper_step_order", ctypes.c_int),
        ("heat_capacity", ctypes.c_double),
        ("T_rad0", _dp),
        ("kappa_full", _dp),
        ("flux", ctypes.c_int),
        ("rusanov_s", ctypes.c_double),
        ("kappa_s_full", _dp),
        ("rand_oversample", ctypes.c_int),
        ("rand_seed", ctypes.c_ulonglong),
        ("hll_beta", ctypes.c_double),
    ]


class TTStats(ctypes.Structure):
    _fields_ = [
        ("steps", ctypes.c_int),
        ("r1", ctypes.c_int),
        ("r2", ctypes.c_int),
        ("max_R1", ctypes.c_int),
        ("max_R2", ctypes.c_int),
        ("nan_flag", ctypes.c_int),
        ("norm", ctypes.c_double),
        ("discarded_rel", ctypes.c_double),
        ("energy", ctypes.c_double),
        ("k_s", ctypes.c_double),
        ("compression", ctypes.c_double),
        ("seconds", ctypes.c_double),
        ("kernel_ms", ctypes.c_double * 10),
        ("kernel_launches", ctypes.c_longlong * 10),
        ("flops", ctypes.c_double * 10),
        ("medium_energy", ctypes.c_double),
        ("sketch_r1", ctypes.c_int),
        ("sketch_r2", ctypes.c_int),
        ("k_s_impl", ctypes.c_double),
        ("direction_space_rounds", ctypes.c_int),
    ]

    def as_dict(self) -> dict:
        d = {f: getattr(self, f) for f, _ in self._fields_[:12]}
        d["kernel_ms"] = dict(zip(KERNEL_CLASSES, list(self.kernel_ms)))
        d["kernel_launches"] = dict(zip(KERNEL_CLASSES, list(self.kernel_launches)))
        d["flops"] = dict(zip(KERNEL_CLASSES, list(self.flops)))
        d["medium_energy"] = self.medium_energy
        d["sketch_r1"], d["sketch_r2"] = self.sketch_r1, self.sketch_r2
        d["k_s_impl"] = self.k_s_impl
        d["direction_space_rounds"] = self.direction_space_rounds
        return d


class TTInternalRanks(ctypes.Structure):
    _fields_ = [
        ("r_nux", ctypes.c_int),
        ("r_xnu", ctypes.c_int),
        ("C_rel_nu", ctypes.c_double),
        ("C_rel_x", ctypes.c_double),
        ("n_sv_nu", ctypes.c_int),
        ("n_sv_x", ctypes.c_int),
    ]


class TTTuning(ctypes.Structure):
    _fields_ = [
        ("project_blocks", ctypes.c_int),
        ("output_blocks", ctypes.c_int),
        ("gram_blocks", ctypes.c_int),
        ("from_cache", ctypes.c_int),
        ("project_ms", ctypes.c_double),
        ("output_ms", ctypes.c_double),
        ("gram_ms", ctypes.c_double),
        ("project_ms_default", ctypes.c_double),
        ("output_ms_default", ctypes.c_double),
        ("gram_ms_default", ctypes.c_double),
    ]

    def as_dict(self) -> dict:
        return {f: getattr(self, f) for f, _ in self._fields_}


class TTError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"tt_transport error {status}: {msg}")
        self.status = status


def _load():
    # PyTorch's HIP runtime must be the one in the process before the library
    # is loaded: both carry the soname libamdhip64.so.7, so whichever is loaded
    # first is used by both, and the library's first HIP call fails if torch
    # later finds a runtime other than its own.
    import torch  # noqa: F401

    if not os.path.exists(LIB_PATH):
        raise ImportError(
            f"{LIB_PATH} is missing: build it with `python -c 'import __graft_entry__ as g; g.build()'` "
            "(hipcc --offload-arch=gfx950); there is no CPU fallback")
    L = ctypes.CDLL(LIB_PATH)
    vp = ctypes.c_void_p
    L.tt_transport_workspace_bytes.argtypes = [ctypes.POINTER(TTProblem)]
    L.tt_transport_workspace_bytes.restype = ctypes.c_size_t
    L.tt_transport_create.argtypes = [ctypes.POINTER(TTProblem), vp, ctypes.c_size_t, vp, ctypes.POINTER(vp)]
    L.tt_transport_create_noalloc.argtypes = [ctypes.POINTER(TTProblem), vp, ctypes.POINTER(vp)]
    L.tt_transport_apply_op.argtypes = [vp, vp]
    L.tt_transport_round.argtypes = [vp, ctypes.c_double, ctypes.c_int, vp]
    L.tt_transport_solve.argtypes = [vp, ctypes.c_int, ctypes.POINTER(TTStats), vp]
    L.tt_transport_reset.argtypes = [vp, vp]
    L.tt_transport_get_ranks.argtypes = [vp, ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_int)]
    L.tt_transport_get_cores.argtypes = [vp, _dp, _dp, _dp, vp]
    L.tt_transport_set_cores.argtypes = [vp, ctypes.c_int, ctypes.c_int, _dp, _dp, _dp, vp]
    L.tt_transport_get_stats.argtypes = [vp, ctypes.POINTER(TTStats)]
    L.tt_transport_set_timing.argtypes = [vp, ctypes.c_int]
    L.tt_transport_set_graph.argtypes = [vp, ctypes.c_int]
    L.tt_transport_tune.argtypes = [vp, ctypes.c_char_p, ctypes.POINTER(TTTuning), vp]
    L.tt_transport_set_launch.argtypes = [vp, ctypes.POINTER(TTTuning)]
    L.tt_transport_get_launch.argtypes = [vp, ctypes.POINTER(TTTuning), ctypes.POINTER(TTTuning)]
    L.tt_transport_step_batch.argtypes = [ctypes.POINTER(vp), ctypes.c_int, ctypes.POINTER(vp), ctypes.c_int]
    L.tt_transport_solve_batch.argtypes = [ctypes.POINTER(vp), ctypes.c_int, ctypes.c_int, ctypes.POINTER(vp),
                                           ctypes.c_int, ctypes.POINTER(TTStats)]
    L.tt_transport_solve_small_batch.argtypes = [ctypes.POINTER(vp), ctypes.c_int, ctypes.POINTER(ctypes.c_int), vp,
                                                 ctypes.POINTER(TTStats)]
    L.tt_transport_destroy.argtypes = [vp]
    L.tt_transport_last_error.argtypes = []
    L.tt_transport_last_error.restype = ctypes.c_char_p
    L.tt_transport_group_emission.argtypes = [_dp, ctypes.c_int, ctypes.c_double, _dp]
    L.tt_transport_get_temperature.argtypes = [vp, _dp, vp]
    L.tt_transport_internal_ranks.argtypes = [vp, ctypes.c_double, ctypes.POINTER(TTInternalRanks), _dp, ctypes.c_int,
                                              _dp, ctypes.c_int, vp]
    for name in ("create", "create_noalloc", "apply_op", "round", "solve", "reset", "get_ranks", "get_cores", "set_cores",
                 "get_stats", "set_timing", "set_graph", "tune", "set_launch", "get_launch", "step_batch", "solve_batch", "solve_small_batch", "destroy",
                 "group_emission",
                 "get_temperature", "internal_ranks"):
        getattr(L, "tt_transport_" + name).restype = ctypes.c_int
    return L


lib = _load()

EXPORTED = ("tt_transport_workspace_bytes", "tt_transport_create", "tt_transport_create_noalloc", "tt_transport_apply_op", "tt_transport_round",
            "tt_transport_solve", "tt_transport_reset", "tt_transport_get_ranks", "tt_transport_get_cores",
            "tt_transport_set_cores", "tt_transport_get_stats", "tt_transport_set_timing", "tt_transport_set_graph",
            "tt_transport_tune", "tt_transport_set_launch", "tt_transport_get_launch",
            "tt_transport_step_batch", "tt_transport_solve_batch", "tt_transport_solve_small_batch",
            "tt_transport_destroy", "tt_transport_last_error",
            "tt_transport_group_emission", "tt_transport_get_temperature", "tt_transport_internal_ranks")


def _check(status: int):
    if status != TT_OK:
        raise TTError(status, lib.tt_transport_last_error().decode())


def _arr(x) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(x, dtype=np.float64))


def group_emission(edges, T: float) -> np.ndarray:
    e = _arr(edges)
    out = np.empty(len(e) - 1)
    _check(lib.tt_transport_group_emission(e.ctypes.data_as(_dp), len(e) - 1, float(T), out.ctypes.data_as(_dp)))
    return out


class ProblemStruct:
    """A tt_problem built from a problem description (attributes as in
    tt_inputs.Problem); keeps the numpy arrays alive while referenced."""

    def __init__(self, prob, round_method: Optional[int] = None):
        self.keep = []

        def ptr(a):
            if a is None:
                return None
            a = _arr(a)
            self.keep.append(a)
            return a.ctypes.data_as(_dp)

        s = TTProblem()
        s.dim = int(prob.dim)
        for d in range(3):
            s.n_cells[d] = int(prob.n_cells[d]) if d < prob.dim else 1
            s.extent[d] = float(prob.extent[d])
        s.n_groups = len(prob.edges) - 1
        s.group_edges = ptr(prob.edges)
        s.kappa0 = ptr(prob.kappa0)
        s.kappa_group_scale = ptr(prob.kappa_scale)
        s.T_cell = ptr(prob.T_cell)
        s.n_theta = len(prob.mu)
        s.n_phi = len(prob.w_phi)
        s.mu = ptr(prob.mu)
        s.w_theta = ptr(prob.w_theta)
        s.phi = ptr(prob.phi)
        s.w_phi = ptr(prob.w_phi)
        for f in range(6):
            s.bc[f] = int(prob.bc[f])
            s.bc_T[f] = float(prob.bc_T[f])
        s.bc_values = ptr(None if prob.bc_values is None else np.asarray(prob.bc_values).reshape(-1))
        s.c = float(prob.c)
        s.cfl = float(prob.cfl)
        s.tol = float(prob.tol)
        s.rank_cap = int(prob.rank_cap)
        s.precision = int(prob.precision)
        s.round_method = int(getattr(prob, "round_method", TT_ROUND_AUTO) if round_method is None else round_method)
        s.paper_step_order = int(prob.step_order)
        s.heat_capacity = float(getattr(prob, "heat_capacity", 0.0))
        s.T_rad0 = ptr(getattr(prob, "T_rad0", None))
        kf = getattr(prob, "kappa_full", None)
        s.kappa_full = ptr(None if kf is None else np.asarray(kf, float).reshape(-1))
        s.flux = int(getattr(prob, "flux", TT_FLUX_UPWIND))
        s.rusanov_s = float(getattr(prob, "rusanov_s", 1.0))
        ks = getattr(prob, "kappa_s_full", None)
        s.kappa_s_full = ptr(None if ks is None else np.asarray(ks, float).reshape(-1))
        s.rand_oversample = int(getattr(prob, "rand_oversample", 4))
        s.rand_seed = int(getattr(prob, "rand_seed", 0))
        s.hll_beta = float(getattr(prob, "hll_beta", 20.0))
        self.s = s


def workspace_bytes(prob, round_method: Optional[int] = None) -> int:
    ps = ProblemStruct(prob, round_method)
    n = lib.tt_transport_workspace_bytes(ctypes.byref(ps.s))
    if n == 0:
        raise TTError(TT_ERR_INVALID_ARG, lib.tt_transport_last_error().decode())
    return int(n)


class Solver:
    """One TT transport solve on a GPU: owns the device workspace (a torch
    uint8 tensor) and the library handle."""

    def __init__(self, prob, device="cuda:0", stream=None, round_method: Optional[int] = None, workspace=None,
                 noalloc: bool = False):
        """noalloc: create with tt_transport_create_noalloc (the library's static
        workspace of its device; nothing is allocated)."""
        import torch

        self.prob = prob
        self.device = torch.device(device)
        self._ps = ProblemStruct(prob, round_method)
        nbytes = lib.tt_transport_workspace_bytes(ctypes.byref(self._ps.s))
        if nbytes == 0:
            _check(TT_ERR_INVALID_ARG)
        self.nbytes = int(nbytes)
        self._stream = stream
        self._noalloc = bool(noalloc)
        self.handle = ctypes.c_void_p()
        if noalloc:
            self.workspace = None
            with torch.cuda.device(self.device):
                _check(lib.tt_transport_create_noalloc(ctypes.byref(self._ps.s), self._sp(), ctypes.byref(self.handle)))
        else:
            if workspace is None:
                workspace = torch.empty(self.nbytes + 256, dtype=torch.uint8, device=self.device)
            self.workspace = workspace
            base = workspace.data_ptr()
            aligned = (base + 255) & ~255
            _check(lib.tt_transport_create(ctypes.byref(self._ps.s), ctypes.c_void_p(aligned),
                                           self.nbytes + 256 - (aligned - base), self._sp(),
                                           ctypes.byref(self.handle)))
        self.M = prob.n_x * (len(prob.edges) - 1)
        self.n_theta = len(prob.mu)
        self.n_phi = len(prob.w_phi)

    def _sp(self):
        import torch

        if self._stream is None:
            return ctypes.c_void_p(torch.cuda.current_stream(self.device).cuda_stream)
        return ctypes.c_void_p(self._stream.cuda_stream)

    # ----- C ABI, same names -----
    def apply_op(self):
        _check(lib.tt_transport_apply_op(self.handle, self._sp()))

    def round(self, tol: float, rank_cap: int):
        _check(lib.tt_transport_round(self.handle, float(tol), int(rank_cap), self._sp()))

    def solve(self, n_steps: int) -> dict:
        st = TTStats()
        _check(lib.tt_transport_solve(self.handle, int(n_steps), ctypes.byref(st), self._sp()))
        return st.as_dict()

    def solve_async(self, n_steps: int):
        """Enqueue n_steps and return after the final synchronisation, no stats."""
        _check(lib.tt_transport_solve(self.handle, int(n_steps), None, self._sp()))

    def reset(self):
        _check(lib.tt_transport_reset(self.handle, self._sp()))

    def get_ranks(self):
        r1, r2 = ctypes.c_int(), ctypes.c_int()
        _check(lib.tt_transport_get_ranks(self.handle, ctypes.byref(r1), ctypes.byref(r2)))
        return r1.value, r2.value

    def get_cores(self, pending_shape=None):
        """Host FP64 copies (Z, Theta, Phi).  For a pending unrounded sum pass
        pending_shape = (R1, R2)."""
        if pending_shape is None:
            r1, r2 = self.get_ranks()
        else:
            r1, r2 = pending_shape
        Z = np.empty((self.M, r1))
        Th = np.empty((r1, self.n_theta, r2))
        Ph = np.empty((r2, self.n_phi))
        _check(lib.tt_transport_get_cores(self.handle, Z.ctypes.data_as(_dp), Th.ctypes.data_as(_dp),
                                          Ph.ctypes.data_as(_dp), self._sp()))
        return Z, Th, Ph

    def set_cores(self, Z, Th, Ph):
        Z, Th, Ph = _arr(Z), _arr(Th), _arr(Ph)
        _check(lib.tt_transport_set_cores(self.handle, Z.shape[1], Ph.shape[0], Z.ctypes.data_as(_dp),
                                          Th.ctypes.data_as(_dp), Ph.ctypes.data_as(_dp), self._sp()))

    def get_temperature(self) -> np.ndarray:
        """Medium temperature per cell (current values when coupled)."""
        T = np.empty(self.prob.n_x)
        _check(lib.tt_transport_get_temperature(self.handle, T.ctypes.data_as(_dp), self._sp()))
        return T

    def internal_ranks(self, delta: float) -> dict:
        """Internal delta-ranks r_nux, r_xnu of the combined core with the
        relative compression ratios and the singular values of both unfoldings."""
        n_groups = self.M // self.prob.n_x
        cap_x = n_groups * max(self.get_ranks()[0], 1)
        sv_nu = np.zeros(n_groups)
        sv_x = np.zeros(cap_x)
        out = TTInternalRanks()
        _check(lib.tt_transport_internal_ranks(self.handle, float(delta), ctypes.byref(out), sv_nu.ctypes.data_as(_dp),
                                               n_groups, sv_x.ctypes.data_as(_dp), cap_x, self._sp()))
        return {"r_nux": out.r_nux, "r_xnu": out.r_xnu, "C_rel_nu": out.C_rel_nu, "C_rel_x": out.C_rel_x,
                "s_nu": sv_nu[:min(out.n_sv_nu, n_groups)], "s_x": sv_x[:min(out.n_sv_x, cap_x)]}

    def get_stats(self) -> dict:
        st = TTStats()
        _check(lib.tt_transport_get_stats(self.handle, ctypes.byref(st)))
        return st.as_dict()

    def set_timing(self, on: bool):
        _check(lib.tt_transport_set_timing(self.handle, 1 if on else 0))

    def set_graph(self, on: bool):
        """Replay the steps of solve() as HIP graphs (needs a non-default stream)."""
        _check(lib.tt_transport_set_graph(self.handle, 1 if on else 0))

    def tune(self, cache_path: Optional[str] = None) -> dict:
        """Time candidate grids of the persistent contraction kernels on the
        current state and keep the fastest (tt_transport_tune)."""
        out = TTTuning()
        path = None if cache_path is None else os.fsencode(cache_path)
        _check(lib.tt_transport_tune(self.handle, path, ctypes.byref(out), self._sp()))
        return out.as_dict()

    def set_launch(self, project_blocks: int = 0, output_blocks: int = 0, gram_blocks: int = 0):
        """Set grid sizes explicitly (0 keeps the current one)."""
        t = TTTuning(project_blocks=int(project_blocks), output_blocks=int(output_blocks),
                     gram_blocks=int(gram_blocks))
        _check(lib.tt_transport_set_launch(self.handle, ctypes.byref(t)))

    def get_launch(self) -> tuple:
        """(current, maximum) grid sizes as dicts."""
        cur, mx = TTTuning(), TTTuning()
        _check(lib.tt_transport_get_launch(self.handle, ctypes.byref(cur), ctypes.byref(mx)))
        keys = ("project_blocks", "output_blocks", "gram_blocks")
        return {k: getattr(cur, k) for k in keys}, {k: getattr(mx, k) for k in keys}

    def destroy(self):
        if self.handle:
            if getattr(self, "_noalloc", False):
                # the static workspace is shared by the next handle on this device:
                # let this handle's work finish first
                import torch
                torch.cuda.synchronize(self.device)
            lib.tt_transport_destroy(self.handle)
            self.handle = ctypes.c_void_p()

    def __del__(self):
        try:
            self.destroy()
        except Exception:
            pass


def _stream_array(streams):
    return (ctypes.c_void_p * len(streams))(*[ctypes.c_void_p(st.cuda_stream) for st in streams])


def step_batch(solvers, streams):
    """One step of every solver; solver i runs on streams[i % len(streams)]."""
    arr = (ctypes.c_void_p * len(solvers))(*[s.handle for s in solvers])
    _check(lib.tt_transport_step_batch(arr, len(solvers), _stream_array(streams), len(streams)))


def solve_batch(solvers, n_steps, streams):
    """n_steps steps of every solver, interleaved across the streams, then a
    synchronisation; returns one stats dict per solver."""
    arr = (ctypes.c_void_p * len(solvers))(*[s.handle for s in solvers])
    stats = (TTStats * len(solvers))()
    _check(lib.tt_transport_solve_batch(arr, len(solvers), int(n_steps), _stream_array(streams), len(streams), stats))
    return [st.as_dict() for st in stats]


def solve_small_batch(solvers, n_steps, stream=None):
    """n_steps[i] steps of solver i (an int applies to all) in the persistent
    ragged small-solve kernel; synchronises; returns one stats dict per solver."""
    import torch
    n = len(solvers)
    if isinstance(n_steps, int):
        n_steps = [n_steps] * n
    arr = (ctypes.c_void_p * n)(*[s.handle for s in solvers])
    steps = (ctypes.c_int * n)(*[int(k) for k in n_steps])
    stats = (TTStats * n)()
    sp = torch.cuda.current_stream().cuda_stream if stream is None else stream.cuda_stream
    _check(lib.tt_transport_solve_small_batch(arr, n, steps, ctypes.c_void_p(sp), stats))
    return [st.as_dict() for st in stats]
