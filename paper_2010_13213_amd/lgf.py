"""Thin ctypes binding of liblgf.so (C ABI in include/lgf.h).

Argument marshalling only: every step of a solve runs in the library's HIP
kernels.  PyTorch supplies device memory (tensors) and streams.  If the
library has not been built the first call raises -- there is no fallback.
"""
import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liblgf.so")

LGF_OK, LGF_E_INVALID, LGF_E_NOMEM, LGF_E_DEVICE, LGF_E_UNSUPPORTED = range(5)
LGF_FP64, LGF_FP32_REFINE = 0, 1
_PREC = {"fp64": LGF_FP64, "fp32_refine": LGF_FP32_REFINE}

EXPORTED = ["lgf_context_create", "lgf_context_destroy", "lgf_context_bytes", "lgf_plan_create",
            "lgf_plan_create_if", "lgf_plan_create_flgf",
            "lgf_problem_check",
            "lgf_plan_destroy", "lgf_plan_workspace_bytes", "lgf_plan_cells", "lgf_plan_field_len",
            "lgf_solve", "lgf_solve_scratch", "lgf_velocity_refresh", "lgf_solve_indicator",
            "lgf_plan_source_blocks", "lgf_solve_batch", "lgf_table_values", "lgf_table_radius",
            "lgf_block_spectrum", "lgf_context_set_timing", "lgf_context_stage_times",
            "lgf_last_error", "lgf_status_string", "lgf_build_id", "lgf_graph_create", "lgf_graph_create_batch", "lgf_graph_launch",
            "lgf_graph_destroy",
            "lgf_context_set_autotune", "lgf_context_save_tuning", "lgf_context_load_tuning",
            "lgf_context_set_mac_method", "lgf_context_set_lattice_passes",
            "lgf_context_tuning_size"]


class LgfError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__("%s: %s" % (_status_name(status), msg))
        self.status = status


class _Level(ctypes.Structure):
    _fields_ = [("n_blocks", ctypes.c_int32), ("block_ijk", ctypes.POINTER(ctypes.c_int32)),
                ("cell_mask", ctypes.POINTER(ctypes.c_uint8))]


class _Problem(ctypes.Structure):
    _fields_ = [("n_levels", ctypes.c_int32), ("nb", ctypes.c_int32), ("dx0", ctypes.c_double),
                ("n_components", ctypes.c_int32), ("precision", ctypes.c_int32),
                ("ne_blocks", ctypes.c_int32), ("levels", ctypes.POINTER(_Level))]


class Report(ctypes.Structure):
    _fields_ = [("device_ms", ctypes.c_double), ("refine_rel_l2", ctypes.c_double),
                ("passes", ctypes.c_int32), ("reserved", ctypes.c_int32)]


_lib = None


def _check_build(bid):
    """The library must have been built from the sources beside it: a stale
    liblgf.so would test and time other code than the tree holds."""
    from . import build as _build
    if not os.path.isdir(_build.CSRC):
        return   # an installed library without its sources: nothing to compare against
    want = "sha256=" + _build.source_digest()
    if not bid.startswith(want + " "):
        raise RuntimeError("liblgf.so (%s) was built from other sources than %s (%s); rebuild with "
                           "python -m paper_2010_13213_amd.build" % (bid, _HERE, want))


def build_id():
    """lgf_build_id() of the loaded library: source digest and target."""
    return lib().lgf_build_id().decode()


def lib():
    """Load liblgf.so; raise if it is missing (no CPU fallback exists)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError("liblgf.so is not built (python -m paper_2010_13213_amd.build); "
                           "the LGF path has no fallback")
    # torch first: its HIP runtime is then the one the process has loaded when
    # the library's own dependency on the runtime is resolved, so both use a
    # single runtime (loading the library first leaves torch without devices)
    import torch  # noqa: F401
    L = ctypes.CDLL(LIB_PATH)
    L.lgf_build_id.argtypes = []
    L.lgf_build_id.restype = ctypes.c_char_p
    _check_build(L.lgf_build_id().decode())
    vp, sz = ctypes.c_void_p, ctypes.c_size_t
    L.lgf_context_create.argtypes = [ctypes.c_int, sz, ctypes.POINTER(vp)]
    L.lgf_context_create.restype = ctypes.c_int
    L.lgf_context_destroy.argtypes = [vp]
    L.lgf_context_destroy.restype = None
    L.lgf_context_bytes.argtypes = [vp]
    L.lgf_context_bytes.restype = sz
    L.lgf_plan_create.argtypes = [vp, ctypes.POINTER(_Problem), ctypes.POINTER(vp)]
    L.lgf_plan_create.restype = ctypes.c_int
    L.lgf_plan_create_if.argtypes = [vp, ctypes.POINTER(_Problem), ctypes.c_double, ctypes.POINTER(vp)]
    L.lgf_plan_create_if.restype = ctypes.c_int
    L.lgf_plan_create_flgf.argtypes = [vp, ctypes.POINTER(_Problem), ctypes.c_int, ctypes.POINTER(vp)]
    L.lgf_plan_create_flgf.restype = ctypes.c_int
    L.lgf_problem_check.argtypes = [ctypes.POINTER(_Problem)]
    L.lgf_problem_check.restype = ctypes.c_int
    L.lgf_plan_destroy.argtypes = [vp]
    L.lgf_plan_destroy.restype = None
    L.lgf_plan_workspace_bytes.argtypes = [vp]
    L.lgf_plan_workspace_bytes.restype = sz
    L.lgf_plan_cells.argtypes = [vp, ctypes.c_int]
    L.lgf_plan_cells.restype = sz
    L.lgf_plan_field_len.argtypes = [vp]
    L.lgf_plan_field_len.restype = sz
    L.lgf_solve.argtypes = [vp, vp, vp, vp, ctypes.POINTER(Report)]
    L.lgf_solve.restype = ctypes.c_int
    L.lgf_solve_scratch.argtypes = [vp, vp, vp, vp]
    L.lgf_solve_scratch.restype = ctypes.c_int
    L.lgf_velocity_refresh.argtypes = [vp, vp, vp, vp, vp]
    L.lgf_velocity_refresh.restype = ctypes.c_int
    L.lgf_solve_indicator.argtypes = [vp, vp, vp, vp, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double)]
    L.lgf_solve_indicator.restype = ctypes.c_int
    L.lgf_plan_source_blocks.argtypes = [vp, ctypes.c_int, ctypes.POINTER(ctypes.c_int32)]
    L.lgf_plan_source_blocks.restype = ctypes.c_int64
    L.lgf_solve_batch.argtypes = [vp, ctypes.c_int, ctypes.POINTER(vp), ctypes.POINTER(vp),
                                  ctypes.POINTER(vp), vp, ctypes.POINTER(Report)]
    L.lgf_solve_batch.restype = ctypes.c_int
    L.lgf_table_values.argtypes = [vp, ctypes.c_int64, ctypes.POINTER(ctypes.c_int32),
                                   ctypes.POINTER(ctypes.c_double)]
    L.lgf_table_values.restype = ctypes.c_int
    L.lgf_table_radius.argtypes = []
    L.lgf_table_radius.restype = ctypes.c_int
    L.lgf_block_spectrum.argtypes = [vp, ctypes.c_int, ctypes.POINTER(ctypes.c_int32),
                                     ctypes.POINTER(ctypes.c_double)]
    L.lgf_block_spectrum.restype = ctypes.c_int
    L.lgf_context_set_mac_method.argtypes = [vp, ctypes.c_int]
    L.lgf_context_set_mac_method.restype = ctypes.c_int
    L.lgf_context_set_lattice_passes.argtypes = [vp, ctypes.c_int]
    L.lgf_context_set_lattice_passes.restype = ctypes.c_int
    L.lgf_context_set_autotune.argtypes = [vp, ctypes.c_int]
    L.lgf_context_set_autotune.restype = ctypes.c_int
    L.lgf_context_save_tuning.argtypes = [vp, ctypes.c_char_p]
    L.lgf_context_save_tuning.restype = ctypes.c_int
    L.lgf_context_load_tuning.argtypes = [vp, ctypes.c_char_p]
    L.lgf_context_load_tuning.restype = ctypes.c_int
    L.lgf_context_tuning_size.argtypes = [vp, ctypes.POINTER(ctypes.c_int64)]
    L.lgf_context_tuning_size.restype = ctypes.c_int
    L.lgf_context_set_timing.argtypes = [vp, ctypes.c_int]
    L.lgf_context_set_timing.restype = ctypes.c_int
    L.lgf_context_stage_times.argtypes = [vp, ctypes.POINTER(ctypes.c_double),
                                          ctypes.POINTER(ctypes.c_int64)]
    L.lgf_context_stage_times.restype = ctypes.c_int
    L.lgf_last_error.argtypes = []
    L.lgf_last_error.restype = ctypes.c_char_p
    L.lgf_status_string.argtypes = [ctypes.c_int]
    L.lgf_status_string.restype = ctypes.c_char_p
    L.lgf_graph_create.argtypes = [vp, vp, vp, ctypes.POINTER(vp)]
    L.lgf_graph_create.restype = ctypes.c_int
    L.lgf_graph_create_batch.argtypes = [vp, ctypes.c_int, ctypes.POINTER(vp), ctypes.POINTER(vp),
                                         ctypes.POINTER(vp), ctypes.POINTER(vp)]
    L.lgf_graph_create_batch.restype = ctypes.c_int
    L.lgf_graph_launch.argtypes = [vp, vp]
    L.lgf_graph_launch.restype = ctypes.c_int
    L.lgf_graph_destroy.argtypes = [vp]
    L.lgf_graph_destroy.restype = None
    _lib = L
    return L


def _status_name(s):
    try:
        return lib().lgf_status_string(s).decode()
    except Exception:
        return "status %d" % s


def _check(status):
    if status != LGF_OK:
        raise LgfError(status, lib().lgf_last_error().decode())


def _stream_handle(stream):
    if stream is None:
        import torch
        return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    if hasattr(stream, "cuda_stream"):
        return ctypes.c_void_p(stream.cuda_stream)
    return ctypes.c_void_p(int(stream))


class Context:
    """Device-resident LGF table and spectra cache on one GPU."""

    def __init__(self, device=0, hbm_budget_bytes=0):
        h = ctypes.c_void_p()
        _check(lib().lgf_context_create(int(device), int(hbm_budget_bytes), ctypes.byref(h)))
        self._h = h
        self.device = int(device)
        self.hbm_budget_bytes = int(hbm_budget_bytes)

    @property
    def handle(self):
        return self._h

    def bytes(self):
        return int(lib().lgf_context_bytes(self._h))

    def close(self):
        if getattr(self, "_h", None):
            lib().lgf_context_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    STAGES = ("fwd_fft", "smac", "inv_fft", "other", "lat_x", "lat_yz", "lat_xinv", "lat_fused")

    MAC_METHODS = {"auto": 0, "pairs": 1, "lattice": 2}

    def set_mac_method(self, method):
        """'auto' (tuning table, else model), 'pairs' or 'lattice' (where the box allows it)."""
        _check(lib().lgf_context_set_mac_method(self._h, self.MAC_METHODS[method]))

    def set_lattice_passes(self, passes):
        """3: the lattice MAC in three passes (default); 1: in one pass per frequency where its lengths are 32^3."""
        _check(lib().lgf_context_set_lattice_passes(self._h, int(passes)))

    def set_autotune(self, reps):
        """Time every compiled MAC tile shape on new convolution shapes (reps > 0) or not (0)."""
        _check(lib().lgf_context_set_autotune(self._h, int(reps)))

    def save_tuning(self, path):
        _check(lib().lgf_context_save_tuning(self._h, str(path).encode()))

    def load_tuning(self, path):
        _check(lib().lgf_context_load_tuning(self._h, str(path).encode()))

    def tuning_size(self):
        n = ctypes.c_int64()
        _check(lib().lgf_context_tuning_size(self._h, ctypes.byref(n)))
        return n.value

    def set_timing(self, enable=True):
        _check(lib().lgf_context_set_timing(self._h, 1 if enable else 0))

    def stage_times(self):
        """{stage: (total_ms, launches)} since the last call; waits for the events."""
        ms = (ctypes.c_double * len(self.STAGES))()
        n = (ctypes.c_int64 * len(self.STAGES))()
        _check(lib().lgf_context_stage_times(self._h, ms, n))
        return {k: (ms[i], n[i]) for i, k in enumerate(self.STAGES)}

    def table_values(self, ijk):
        ijk = np.ascontiguousarray(ijk, dtype=np.int32).reshape(-1, 3)
        out = np.empty(len(ijk))
        _check(lib().lgf_table_values(self._h, len(ijk),
                                      ijk.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                                      out.ctypes.data_as(ctypes.POINTER(ctypes.c_double))))
        return out

    def block_spectrum(self, nb, d):
        d = np.ascontiguousarray(d, dtype=np.int32).reshape(3)
        N = 2 * nb
        out = np.empty(2 * N * N * (nb + 1))
        _check(lib().lgf_block_spectrum(self._h, int(nb),
                                        d.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                                        out.ctypes.data_as(ctypes.POINTER(ctypes.c_double))))
        return (out[0::2] + 1j * out[1::2]).reshape(N, N, nb + 1)


def table_radius():
    return int(lib().lgf_table_radius())


def _problem(level_blocks, nb, dx0, n_components, precision, ne_blocks, cell_masks=None):
    blocks = [np.ascontiguousarray(b, dtype=np.int32).reshape(-1, 3) for b in level_blocks]
    masks = [None if m is None else np.ascontiguousarray(m, dtype=np.uint8).reshape(-1)
             for m in (cell_masks or [None] * len(blocks))]
    levels = (_Level * max(1, len(blocks)))()
    for i, b in enumerate(blocks):
        levels[i].n_blocks = len(b)
        levels[i].block_ijk = b.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))
        if masks[i] is not None:
            if masks[i].size != len(b) * int(nb) ** 3:
                raise ValueError("cell mask of level %d needs %d bytes" % (i, len(b) * int(nb) ** 3))
            levels[i].cell_mask = masks[i].ctypes.data_as(ctypes.POINTER(ctypes.c_uint8))
    prob = _Problem(len(blocks), int(nb), float(dx0), int(n_components),
                    _PREC[precision] if isinstance(precision, str) else int(precision),
                    int(ne_blocks), levels)
    return prob, (blocks, masks, levels)


def problem_check(level_blocks, nb, dx0, n_components=1, precision="fp64", ne_blocks=0, cell_masks=None):
    """Host-only validation of a problem; returns (status, message)."""
    prob, keep = _problem(level_blocks, nb, dx0, n_components, precision, ne_blocks, cell_masks)
    st = lib().lgf_problem_check(ctypes.byref(prob))
    return st, (lib().lgf_last_error().decode() if st != LGF_OK else "")


class Plan:
    """An immutable solve plan for one block support (all levels)."""

    def __init__(self, ctx, level_blocks, nb, dx0, n_components=1, precision="fp64", ne_blocks=0, if_a0=None,
                 cell_masks=None, flgf_near=None):
        """if_a0: None for the LGF solve (L^-1); a > 0 for the integrating
        factor H(a) = exp(a L) on level 0 (a_k = 4^k a on level k).
        cell_masks: None or one entry per level, None or nb^3 bytes per
        block ([block][z][y][x]; 1 keeps the cell in Omega_k).
        flgf_near: None for the exact sum; D >= 0 for the two-grid fast-LGF
        approximation with block pairs within D blocks summed exactly."""
        self.ctx = ctx
        self.nb = int(nb)
        self.n_levels = len(level_blocks)
        self.n_components = int(n_components)
        self.precision = precision
        prob, self._keep = _problem(level_blocks, nb, dx0, n_components, precision, ne_blocks, cell_masks)
        h = ctypes.c_void_p()
        if flgf_near is not None:
            _check(lib().lgf_plan_create_flgf(ctx.handle, ctypes.byref(prob), int(flgf_near), ctypes.byref(h)))
        elif if_a0 is None:
            _check(lib().lgf_plan_create(ctx.handle, ctypes.byref(prob), ctypes.byref(h)))
        else:
            _check(lib().lgf_plan_create_if(ctx.handle, ctypes.byref(prob), float(if_a0), ctypes.byref(h)))
        self._h = h

    @classmethod
    def for_problem(cls, ctx, problem, precision="fp64", ne_blocks=0, if_a0=None, flgf_near=None):
        masks = [getattr(lv, "cell_mask", None) for lv in problem.levels]
        return cls(ctx, [lv.blocks for lv in problem.levels], problem.nb, problem.dx0,
                   problem.n_components, precision, ne_blocks, if_a0,
                   None if all(m is None for m in masks) else masks, flgf_near)

    @property
    def handle(self):
        return self._h

    def field_len(self):
        return int(lib().lgf_plan_field_len(self._h))

    def cells(self, level=0):
        return int(lib().lgf_plan_cells(self._h, int(level)))

    def workspace_bytes(self):
        return int(lib().lgf_plan_workspace_bytes(self._h))

    def close(self):
        if getattr(self, "_h", None):
            lib().lgf_plan_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def solve(self, f, u=None, stream=None, report=False):
        """u = LGF solve of f (CUDA float64 tensors of field_len() elements)."""
        import torch
        n = self.field_len()
        if f.dtype != torch.float64 or not f.is_cuda or f.numel() != n or not f.is_contiguous():
            raise ValueError("f must be a contiguous CUDA float64 tensor of %d elements" % n)
        if u is None:
            u = torch.empty_like(f)
        rep = Report() if report else None
        _check(lib().lgf_solve(self._h, ctypes.c_void_p(f.data_ptr()), ctypes.c_void_p(u.data_ptr()),
                               _stream_handle(stream), ctypes.byref(rep) if rep is not None else None))
        return (u, rep) if report else u

    def source_blocks(self, level):
        """Blocks of the level's combined source R_k ((n, 3) int32)."""
        n = int(lib().lgf_plan_source_blocks(self._h, int(level), None))
        if n < 0:
            raise ValueError("no level %d" % level)
        out = np.empty((n, 3), dtype=np.int32)
        lib().lgf_plan_source_blocks(self._h, int(level), out.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)))
        return out

    def solve_indicator(self, f, u=None, stream=None):
        """lgf_solve_indicator: returns (u, rms, max), rms / max as lists per
        component of lists per level of per-block arrays."""
        import torch
        n = self.field_len()
        _check_field(f, n, "f")
        u = torch.empty_like(f) if u is None else u
        _check_field(u, n, "u")
        counts = [len(self.source_blocks(k)) for k in range(self.n_levels)]
        tot = sum(counts) * self.n_components
        rms = np.empty(tot)
        mx = np.empty(tot)
        dp = ctypes.POINTER(ctypes.c_double)
        _check(lib().lgf_solve_indicator(self._h, ctypes.c_void_p(f.data_ptr()), ctypes.c_void_p(u.data_ptr()),
                                         _stream_handle(stream), rms.ctypes.data_as(dp), mx.ctypes.data_as(dp)))
        split = np.cumsum(counts)[:-1]
        per = lambda a: [np.split(r, split) for r in a.reshape(self.n_components, -1)]
        return u, per(rms), per(mx)

    def solve_scratch(self, f, u, stream=None):
        """lgf_solve_scratch: the same solve with the spectral workspace in the
        library's static device array (allocates nothing; u must be given)."""
        import torch
        n = self.field_len()
        for t in (f, u):
            if t.dtype != torch.float64 or not t.is_cuda or t.numel() != n or not t.is_contiguous():
                raise ValueError("f and u must be contiguous CUDA float64 tensors of %d elements" % n)
        _check(lib().lgf_solve_scratch(self._h, ctypes.c_void_p(f.data_ptr()), ctypes.c_void_p(u.data_ptr()),
                                       _stream_handle(stream)))
        return u


def _check_field(t, n, name):
    import torch
    if t.dtype != torch.float64 or not t.is_cuda or t.numel() != n or not t.is_contiguous():
        raise ValueError("%s must be a contiguous CUDA float64 tensor of %d elements" % (name, n))


def velocity_refresh(plan, omega, psi=None, u=None, stream=None):
    """lgf_velocity_refresh: u = -C^dagger L_E^-1 omega on a single-level
    3-component plan; returns (psi, u)."""
    import torch
    n = plan.field_len()
    _check_field(omega, n, "omega")
    psi = torch.empty_like(omega) if psi is None else psi
    u = torch.empty_like(omega) if u is None else u
    _check_field(psi, n, "psi")
    _check_field(u, n, "u")
    _check(lib().lgf_velocity_refresh(plan.handle, ctypes.c_void_p(omega.data_ptr()), ctypes.c_void_p(psi.data_ptr()),
                                      ctypes.c_void_p(u.data_ptr()), _stream_handle(stream)))
    return psi, u


def scratch_max_bytes():
    """LGF_SCRATCH_MAX_BYTES of include/lgf.h: the static scratch of lgf_solve_scratch."""
    return 64 << 20


class Graph:
    """One solve of `plan` on the fixed tensors f, u, captured as a HIP graph
    (lgf_graph_create); launch() replays it.  Keep f, u and the plan alive
    while the graph exists."""

    def __init__(self, plan, f, u):
        import torch
        n = plan.field_len()
        for t in (f, u):
            if t.dtype != torch.float64 or not t.is_cuda or t.numel() != n or not t.is_contiguous():
                raise ValueError("f and u must be contiguous CUDA float64 tensors of %d elements" % n)
        self.plan, self.f, self.u = plan, f, u
        self._h = ctypes.c_void_p()
        _check(lib().lgf_graph_create(plan.handle, ctypes.c_void_p(f.data_ptr()), ctypes.c_void_p(u.data_ptr()),
                                      ctypes.byref(self._h)))

    def launch(self, stream=None):
        _check(lib().lgf_graph_launch(self._h, _stream_handle(stream)))
        return self.u

    def close(self):
        if self._h:
            lib().lgf_graph_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class BatchGraph:
    """One lgf_solve_batch of `plans` on the fixed tensors fs, us, captured
    as a HIP graph (lgf_graph_create_batch); launch() replays it.  Keep the
    plans, tensors and context alive while the graph exists."""

    def __init__(self, ctx, plans, fs, us):
        n = len(plans)
        for p, f, u in zip(plans, fs, us):
            _check_field(f, p.field_len(), "f")
            _check_field(u, p.field_len(), "u")
        self.ctx, self.plans, self.fs, self.us = ctx, list(plans), list(fs), list(us)
        P = (ctypes.c_void_p * n)(*[p.handle.value for p in plans])
        F = (ctypes.c_void_p * n)(*[f.data_ptr() for f in fs])
        U = (ctypes.c_void_p * n)(*[u.data_ptr() for u in us])
        self._h = ctypes.c_void_p()
        _check(lib().lgf_graph_create_batch(ctx.handle, n, P, F, U, ctypes.byref(self._h)))

    def launch(self, stream=None):
        _check(lib().lgf_graph_launch(self._h, _stream_handle(stream)))
        return self.us

    def close(self):
        if self._h:
            lib().lgf_graph_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def solve_batch(ctx, plans, fs, us, stream=None, report=False):
    n = len(plans)
    P = (ctypes.c_void_p * n)(*[p.handle.value for p in plans])
    F = (ctypes.c_void_p * n)(*[f.data_ptr() for f in fs])
    U = (ctypes.c_void_p * n)(*[u.data_ptr() for u in us])
    reps = (Report * n)() if report else None
    _check(lib().lgf_solve_batch(ctx.handle, n, P, F, U, _stream_handle(stream), reps))
    return list(reps) if report else None
