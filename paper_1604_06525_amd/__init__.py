"""Python binding of the MI355X matrix-free GN/LM least-squares library (libopt.so).

Argument marshalling only: every step of a solve runs in the HIP kernels of
``libopt.so``; this module turns torch tensors into device pointers and calls
the C ABI of ``include/opt.h`` with the same names.  The first call raises if the
library has not been built (``__graft_entry__.build()`` or
``python -m paper_1604_06525_amd.build``); there is no fallback.
"""
import ctypes
import os

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libopt.so")

OPT_OK, OPT_EINVAL, OPT_ENOMEM, OPT_EHIP, OPT_EAGAIN, OPT_ENUMERIC, OPT_EUNSUPPORTED = 0, -1, -2, -3, -4, -5, -6
GRID2D, GRAPH, GRID3D = 0, 1, 2
ENERGIES = {"laplacian": 0, "arap_warp": 1, "poisson": 2, "sfs": 3, "flow": 4, "arap_mesh": 5, "arap_volume": 6,
            "lp_smooth": 7, "intrinsic": 8}
PRECISIONS = {"fp64": 0, "mixed": 1}
GN, LM = 0, 1
PCG_FUSED, PCG_SPLIT, PCG_MATERIALIZED, PCG_RECOMPUTE = 0, 1, 2, 3


class opt_problem_desc(ctypes.Structure):
    _fields_ = [("domain", ctypes.c_int32), ("energy", ctypes.c_int32), ("precision", ctypes.c_int32),
                ("width", ctypes.c_int32), ("height", ctypes.c_int32),
                ("n_vertices", ctypes.c_int32), ("n_edges", ctypes.c_int32),
                ("edges", ctypes.c_void_p), ("arrays", ctypes.c_void_p * 8),
                ("params", ctypes.c_double * 16), ("n_params", ctypes.c_int32), ("depth", ctypes.c_int32),
                ("materialize", ctypes.c_int32)]


class opt_solve_params(ctypes.Structure):
    _fields_ = [("method", ctypes.c_int32), ("outer_iters", ctypes.c_int32),
                ("pcg_iters", ctypes.c_int32), ("use_precond", ctypes.c_int32),
                ("lm_radius0", ctypes.c_double), ("lm_radius_min", ctypes.c_double),
                ("lm_radius_max", ctypes.c_double), ("lm_diag_min", ctypes.c_double),
                ("lm_diag_max", ctypes.c_double), ("lm_min_rel_decrease", ctypes.c_double),
                ("pcg_variant", ctypes.c_int32)]


class opt_tuning(ctypes.Structure):
    _fields_ = [("strip_rows", ctypes.c_int32), ("waves_per_simd", ctypes.c_int32),
                ("large_grid_form", ctypes.c_int32)]


class opt_solve_report(ctypes.Structure):
    _fields_ = [("cost_initial", ctypes.c_double), ("cost_final", ctypes.c_double),
                ("outer_done", ctypes.c_int32), ("steps_accepted", ctypes.c_int32),
                ("cost_trace", ctypes.POINTER(ctypes.c_double))]


_P = ctypes.c_void_p
_proto = {
    "opt_last_error": (ctypes.c_char_p, []),
    "opt_workspace_size": (ctypes.c_int, [ctypes.POINTER(opt_problem_desc), ctypes.POINTER(ctypes.c_size_t)]),
    "opt_problem_create": (ctypes.c_int, [ctypes.POINTER(opt_problem_desc), _P, ctypes.c_size_t, _P,
                                          ctypes.POINTER(_P)]),
    "opt_problem_destroy": (ctypes.c_int, [_P]),
    "opt_default_params": (None, [ctypes.POINTER(opt_solve_params)]),
    "opt_solve": (ctypes.c_int, [_P, _P, ctypes.POINTER(opt_solve_params), ctypes.POINTER(opt_solve_report)]),
    "opt_solve_scratch": (ctypes.c_int, [ctypes.POINTER(opt_problem_desc), _P, ctypes.POINTER(opt_solve_params),
                                         ctypes.POINTER(opt_solve_report), _P]),
    "opt_cost": (ctypes.c_int, [_P, _P, ctypes.POINTER(ctypes.c_double)]),
    "opt_linearize": (ctypes.c_int, [_P, _P, ctypes.POINTER(ctypes.c_double)]),
    "opt_eval_jtf": (ctypes.c_int, [_P, _P, _P]),
    "opt_apply_jtj": (ctypes.c_int, [_P, _P, _P, ctypes.c_double, ctypes.POINTER(opt_solve_params)]),
    "opt_pcg": (ctypes.c_int, [_P, ctypes.POINTER(opt_solve_params), ctypes.c_double, _P]),
    "opt_energy_channels": (ctypes.c_int, [ctypes.c_int32]),
    "opt_image_downsample2": (ctypes.c_int, [_P, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                                             _P, _P]),
    "opt_image_gradient": (ctypes.c_int, [_P, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, _P, _P, _P]),
    "opt_field_upsample": (ctypes.c_int, [_P, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                                          ctypes.POINTER(ctypes.c_double), ctypes.c_int32, _P, ctypes.c_int32,
                                          ctypes.c_int32, _P]),
    "opt_flow_pyramid_workspace_size": (ctypes.c_int, [ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                                                       ctypes.c_int32, ctypes.POINTER(ctypes.c_size_t)]),
    "opt_solve_flow_pyramid": (ctypes.c_int, [_P, _P, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                                              ctypes.c_double, ctypes.c_double, ctypes.c_int32,
                                              ctypes.POINTER(opt_solve_params), _P, _P, ctypes.c_size_t, _P,
                                              ctypes.POINTER(opt_solve_report)]),
    "opt_profile_enable": (ctypes.c_int, [_P, ctypes.c_int]),
    "opt_profile_read": (ctypes.c_int, [_P, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int64)]),
    "opt_problem_set_tuning": (ctypes.c_int, [_P, ctypes.POINTER(opt_tuning)]),
    "opt_problem_get_tuning": (ctypes.c_int, [_P, ctypes.POINTER(opt_tuning)]),
    "opt_problem_set_graph_replay": (ctypes.c_int, [_P, ctypes.c_int]),
    "opt_problem_pcg_form": (ctypes.c_int, [_P, ctypes.c_int, ctypes.POINTER(ctypes.c_int)]),
    "opt_server_reserved_bytes": (ctypes.c_int, [ctypes.c_int32, ctypes.POINTER(ctypes.c_size_t)]),
    "opt_server_create": (ctypes.c_int, [_P, ctypes.c_size_t, ctypes.c_int32, _P, ctypes.POINTER(_P)]),
    "opt_server_destroy": (ctypes.c_int, [_P]),
    "opt_server_submit": (ctypes.c_int, [_P, ctypes.POINTER(opt_problem_desc), _P,
                                         ctypes.POINTER(opt_solve_params), ctypes.POINTER(ctypes.c_int64)]),
    "opt_server_step": (ctypes.c_int, [_P]),
    "opt_server_wait": (ctypes.c_int, [_P]),
    "opt_server_set_fill_budget": (ctypes.c_int, [_P, ctypes.c_double]),
    "opt_server_poll": (ctypes.c_int, [_P, ctypes.c_int64, ctypes.POINTER(ctypes.c_int32),
                                       ctypes.POINTER(opt_solve_report)]),
    "opt_server_cancel": (ctypes.c_int, [_P, ctypes.c_int64]),
    "opt_server_info": (ctypes.c_int, [_P, ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_size_t)]),
    "opt_server_add_tuning": (ctypes.c_int, [_P, ctypes.c_int32, ctypes.c_int32, ctypes.c_int64, ctypes.c_int64,
                                             ctypes.POINTER(opt_tuning)]),
}
_lib = None


def lib():
    """The loaded libopt.so; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build the HIP library first "
                              "(python -m paper_1604_06525_amd.build)")
        h = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in _proto.items():
            f = getattr(h, name)
            f.restype = res
            f.argtypes = args
        _lib = h
    return _lib


class OptError(RuntimeError):
    def __init__(self, code, where):
        self.code = code
        msg = lib().opt_last_error().decode(errors="replace")
        super().__init__(f"{where} returned {code}: {msg}")


def _check(code, where):
    if code != OPT_OK:
        raise OptError(code, where)


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else ctypes.c_void_p(0)


def default_params(**kw):
    p = opt_solve_params()
    lib().opt_default_params(ctypes.byref(p))
    for k, v in kw.items():
        if k == "method" and isinstance(v, str):
            v = {"gn": GN, "lm": LM}[v.lower()]
        if k == "pcg_variant" and isinstance(v, str):
            v = {"fused": PCG_FUSED, "split": PCG_SPLIT, "materialized": PCG_MATERIALIZED,
                 "recompute": PCG_RECOMPUTE}[v.lower()]
        if not hasattr(p, k):
            raise TypeError(f"unknown solve parameter {k}")
        setattr(p, k, v)
    return p


def energy_channels(energy):
    return lib().opt_energy_channels(ENERGIES[energy] if isinstance(energy, str) else energy)


# The data arrays each energy takes (include/opt.h): planes over the sites, and
# whether an array holds bulk values (the precision's float type) or a uint8 mask.
ARRAY_SPEC = {
    "arap_warp": [(2, "bulk"), (2, "bulk"), (1, "u8")],
    "poisson": [(4, "bulk"), (1, "u8")],
    "sfs": [(1, "bulk"), (1, "bulk"), (1, "u8"), (1, "u8")],
    "flow": [(1, "bulk"), (1, "bulk"), (1, "bulk"), (1, "bulk")],
    "arap_mesh": [(3, "bulk"), (3, "bulk")],
    "arap_volume": [(3, "bulk"), (3, "bulk")],
    "laplacian": [(1, "bulk")],  # 3 planes on a graph
    "lp_smooth": [(1, "bulk")],
    "intrinsic": [(3, "bulk")],
}


def _check_tensor(t, dtype, numel, what):
    if not isinstance(t, torch.Tensor):
        raise ValueError(f"{what} must be a torch tensor, got {type(t).__name__}")
    if t.dtype != dtype:
        raise ValueError(f"{what} must have dtype {dtype}, got {t.dtype}")
    if t.numel() != numel:
        raise ValueError(f"{what} must have {numel} elements, got {t.numel()}")
    if not t.is_contiguous():
        raise ValueError(f"{what} must be contiguous")


def len_channels(energy, graph=False):
    """Unknown channels per site (the header's table; no library call).  The
    Laplacian smooths a scalar on a grid and a float3 on a graph."""
    if energy == "laplacian":
        return 3 if graph else 1
    return {"arap_warp": 3, "poisson": 4, "sfs": 1, "flow": 2, "arap_mesh": 6, "arap_volume": 6,
            "lp_smooth": 1, "intrinsic": 4}[energy]


def check_request(energy, arrays, x, precision, n_sites, graph=False):
    """Raise ValueError unless the data arrays and the unknowns match what the
    library will read and write for this energy, precision and site count
    (checked on the host before any pointer reaches a kernel)."""
    bulk = torch.float64 if precision == "fp64" else torch.float32
    spec = ARRAY_SPEC.get(energy)
    if spec is None:
        raise ValueError(f"unknown energy {energy}")
    if len(arrays) != len(spec):
        raise ValueError(f"{energy} takes {len(spec)} arrays, got {len(arrays)}")
    if energy == "laplacian" and graph:
        spec = [(3, "bulk")]
    named = [(f"array {k} of {energy}", a) for k, a in enumerate(arrays)]
    for (what, a), (planes, kind) in zip(named, spec):
        _check_tensor(a, bulk if kind == "bulk" else torch.uint8, planes * n_sites, what)
    if x is not None:
        _check_tensor(x, bulk, len_channels(energy, graph) * n_sites, "unknowns")
        named.append(("unknowns", x))
    for what, t in named:
        if t.device.type != "cuda":
            raise ValueError(f"{what} must be on a CUDA device, got {t.device}")


def make_desc(energy, arrays, params=(), precision="mixed", width=0, height=0, n_vertices=0,
              edges=None, depth=0, materialize=False):
    """An opt_problem_desc for the given tensors; returns (desc, arrays, edges)
    (the tensors the descriptor points to, to be kept alive by the caller).
    A graph when n_vertices is given, a 3D grid when depth is, else a 2D grid."""
    d = opt_problem_desc()
    d.domain = GRAPH if n_vertices else (GRID3D if depth else GRID2D)
    d.energy = ENERGIES[energy]
    d.precision = PRECISIONS[precision]
    d.width, d.height = width, height
    d.depth = depth
    d.materialize = int(bool(materialize))
    d.n_vertices = n_vertices
    if edges is not None:
        if not edges.is_contiguous() or edges.dtype != torch.int32:
            raise ValueError("edges must be a contiguous int32 tensor of E x 2")
        d.n_edges = int(edges.shape[0])
        d.edges = edges.data_ptr()
    arrays = list(arrays)
    for k, a in enumerate(arrays):
        if not a.is_contiguous():
            raise ValueError(f"array {k} must be contiguous")
        d.arrays[k] = a.data_ptr()
    params = list(params)
    for k, v in enumerate(params):
        d.params[k] = float(v)
    d.n_params = len(params)
    return d, arrays, edges


class Problem:
    """One problem instance: a grid or graph, an energy and its data arrays.

    ``arrays`` are device tensors in the energy's order (include/opt.h); float64
    under precision "fp64", float32 under "mixed", uint8 for masks.  They are
    referenced, not copied, and kept alive by this object.  The workspace is a
    torch uint8 tensor on the same device.  ``tuning``: "auto" takes the launch
    shape from the committed tuning table (the library's own choice where it has
    no entry), "served" the shape a Server gives the same request, a dict sets
    one by hand, None keeps the library's choice.
    """

    def __init__(self, energy, arrays, params=(), precision="mixed", width=0, height=0,
                 n_vertices=0, edges=None, stream=None, workspace=None, tuning="auto", depth=0,
                 materialize=False):
        self.energy = energy
        self.precision = precision
        self.dtype = torch.float64 if precision == "fp64" else torch.float32
        self.channels = len_channels(energy, bool(n_vertices)) if energy == "laplacian" else energy_channels(energy)
        self.n_sites = n_vertices if n_vertices else width * height * (depth if depth else 1)
        check_request(energy, list(arrays), None, precision, self.n_sites, bool(n_vertices))
        self.desc, self.arrays, self.edges = make_desc(energy, arrays, params, precision, width, height,
                                                       n_vertices, edges, depth, materialize)
        d = self.desc
        nbytes = ctypes.c_size_t(0)
        _check(lib().opt_workspace_size(ctypes.byref(d), ctypes.byref(nbytes)), "opt_workspace_size")
        dev = self.arrays[0].device
        self.device = dev
        if workspace is None:
            workspace = torch.empty(nbytes.value, dtype=torch.uint8, device=dev)
        elif workspace.numel() < nbytes.value or workspace.dtype != torch.uint8:
            raise ValueError(f"workspace must be a uint8 tensor of at least {nbytes.value} bytes")
        self.workspace = workspace
        self.stream = stream if stream is not None else torch.cuda.current_stream(dev)
        h = ctypes.c_void_p(0)
        _check(lib().opt_problem_create(ctypes.byref(d), _ptr(self.workspace), self.workspace.numel(),
                                       ctypes.c_void_p(self.stream.cuda_stream), ctypes.byref(h)),
               "opt_problem_create")
        self.handle = h
        self._lib = lib()
        if tuning in ("auto", "served") and not n_vertices and not depth:
            from . import tune
            t = tune.best(tune.load(), energy, precision, self.n_sites, served=tuning == "served")
            if t["strip_rows"] or t["waves_per_simd"]:
                self.set_tuning(**t)
        elif isinstance(tuning, dict):
            self.set_tuning(**tuning)

    def __del__(self):
        # at interpreter exit the module globals may already be gone; the
        # library handle kept on the instance still works
        h = getattr(self, "handle", None)
        L = getattr(self, "_lib", None)
        if h is not None and h.value and L is not None:
            L.opt_problem_destroy(h)
            self.handle = None

    def _vec(self, t, name):
        shape = (self.channels, self.n_sites)
        if t.dtype != self.dtype or not t.is_contiguous() or t.numel() != shape[0] * shape[1]:
            raise ValueError(f"{name} must be a contiguous {self.dtype} tensor of {shape[0]}x{shape[1]}")
        return t

    def new_vector(self):
        return torch.zeros((self.channels, self.n_sites), dtype=self.dtype, device=self.device)

    def solve(self, x, params=None, report=True, **kw):
        """opt_solve on x (in place).  Returns a dict with the report, or None."""
        self._vec(x, "x")
        self._lin_x = None
        p = params if params is not None else default_params(**kw)
        if not report:
            _check(lib().opt_solve(self.handle, _ptr(x), ctypes.byref(p), None), "opt_solve")
            return None
        trace = (ctypes.c_double * (p.outer_iters + 1))()
        rep = opt_solve_report()
        rep.cost_trace = ctypes.cast(trace, ctypes.POINTER(ctypes.c_double))
        code = lib().opt_solve(self.handle, _ptr(x), ctypes.byref(p), ctypes.byref(rep))
        out = dict(cost_initial=rep.cost_initial, cost_final=rep.cost_final,
                   outer_done=rep.outer_done, steps_accepted=rep.steps_accepted,
                   cost_trace=list(trace), code=code)
        _check(code, "opt_solve")
        return out

    def cost(self, x):
        self._vec(x, "x")
        c = ctypes.c_double(0)
        _check(lib().opt_cost(self.handle, _ptr(x), ctypes.byref(c)), "opt_cost")
        return c.value

    def linearize(self, x, want_cost=True):
        """opt_linearize.  eval_jtf/apply_jtj/pcg read x again later, so the
        tensor is kept alive here until the next linearize or solve."""
        self._vec(x, "x")
        self._lin_x = x
        if not want_cost:
            _check(lib().opt_linearize(self.handle, _ptr(x), None), "opt_linearize")
            return None
        c = ctypes.c_double(0)
        _check(lib().opt_linearize(self.handle, _ptr(x), ctypes.byref(c)), "opt_linearize")
        return c.value

    def eval_jtf(self):
        b, d = self.new_vector(), self.new_vector()
        _check(lib().opt_eval_jtf(self.handle, _ptr(b), _ptr(d)), "opt_eval_jtf")
        return b, d

    def apply_jtj(self, p, lam=0.0, params=None):
        self._vec(p, "p")
        q = self.new_vector()
        prm = params if params is not None else default_params()
        _check(lib().opt_apply_jtj(self.handle, _ptr(p), _ptr(q), float(lam), ctypes.byref(prm)),
               "opt_apply_jtj")
        return q

    def set_tuning(self, strip_rows=0, waves_per_simd=0, large_grid_form=0):
        t = opt_tuning()
        t.strip_rows = int(strip_rows)
        t.waves_per_simd = int(waves_per_simd)
        t.large_grid_form = int(large_grid_form)
        _check(lib().opt_problem_set_tuning(self.handle, ctypes.byref(t)), "opt_problem_set_tuning")

    def get_tuning(self):
        """The launch shape in force: strip_rows and waves_per_simd (resolved),
        plus large_grid_form when it was asked for."""
        t = opt_tuning()
        _check(lib().opt_problem_get_tuning(self.handle, ctypes.byref(t)), "opt_problem_get_tuning")
        out = {"strip_rows": t.strip_rows, "waves_per_simd": t.waves_per_simd}
        if t.large_grid_form:
            out["large_grid_form"] = 1
        return out

    def set_graph_replay(self, on=True):
        """opt_problem_set_graph_replay: replay repeated solves as one HIP graph."""
        _check(lib().opt_problem_set_graph_replay(self.handle, int(on)), "opt_problem_set_graph_replay")

    def pcg_form(self, variant="fused"):
        """opt_problem_pcg_form: the form ("fused", "split", "materialized" or
        "recompute") a solve asking for `variant` runs."""
        v = {"fused": PCG_FUSED, "split": PCG_SPLIT, "materialized": PCG_MATERIALIZED,
                 "recompute": PCG_RECOMPUTE}[variant.lower()]
        out = ctypes.c_int(-1)
        _check(lib().opt_problem_pcg_form(self.handle, v, ctypes.byref(out)), "opt_problem_pcg_form")
        return {PCG_FUSED: "fused", PCG_SPLIT: "split", PCG_MATERIALIZED: "materialized",
                PCG_RECOMPUTE: "recompute"}[out.value]

    def profile_enable(self, on=True):
        _check(lib().opt_profile_enable(self.handle, int(on)), "opt_profile_enable")

    def profile_read(self):
        """(milliseconds, PCG iterations) of the PCG phases timed since the last read."""
        ms = ctypes.c_double(0)
        it = ctypes.c_int64(0)
        _check(lib().opt_profile_read(self.handle, ctypes.byref(ms), ctypes.byref(it)), "opt_profile_read")
        return ms.value, it.value

    def pcg(self, iters, lam=0.0, use_precond=True, params=None, variant="fused"):
        prm = params if params is not None else default_params(
            pcg_iters=iters, use_precond=int(use_precond), pcg_variant=variant)
        d = self.new_vector()
        _check(lib().opt_pcg(self.handle, ctypes.byref(prm), float(lam), _ptr(d)), "opt_pcg")
        return d


SCRATCH_BYTES = 128 << 20  # OPT_SCRATCH_BYTES


def solve_scratch(energy, arrays, x, params=(), precision="mixed", width=0, height=0, n_vertices=0,
                  edges=None, solve_params=None, stream=None, report=True, depth=0, **kw):
    """opt_solve_scratch: create and solve a problem in the library's static
    scratch (no device allocation), x in place.  Returns the report dict (as
    Problem.solve), or None with report=False (work only enqueued)."""
    n = n_vertices if n_vertices else width * height * (depth if depth else 1)
    check_request(energy, list(arrays), x, precision, n, bool(n_vertices))
    d, arrays, edges = make_desc(energy, arrays, params, precision, width, height, n_vertices, edges, depth)
    p = solve_params if solve_params is not None else default_params(**kw)
    st = stream if stream is not None else torch.cuda.current_stream(x.device)
    sp = ctypes.c_void_p(st.cuda_stream)
    if not report:
        _check(lib().opt_solve_scratch(ctypes.byref(d), _ptr(x), ctypes.byref(p), None, sp), "opt_solve_scratch")
        return None
    trace = (ctypes.c_double * (p.outer_iters + 1))()
    rep = opt_solve_report()
    rep.cost_trace = ctypes.cast(trace, ctypes.POINTER(ctypes.c_double))
    code = lib().opt_solve_scratch(ctypes.byref(d), _ptr(x), ctypes.byref(p), ctypes.byref(rep), sp)
    out = dict(cost_initial=rep.cost_initial, cost_final=rep.cost_final,
               outer_done=rep.outer_done, steps_accepted=rep.steps_accepted,
               cost_trace=list(trace), code=code)
    _check(code, "opt_solve_scratch")
    return out


# ---------------------------------------------------------------- multi-pass steps
def _stream_of(t, stream):
    st = stream if stream is not None else torch.cuda.current_stream(t.device)
    return ctypes.c_void_p(st.cuda_stream)


def _img_check(t, precision, numel, name):
    dtype = torch.float64 if precision == "fp64" else torch.float32
    if t.dtype != dtype or not t.is_contiguous() or t.numel() != numel or t.device.type != "cuda":
        raise ValueError(f"{name} must be a contiguous {dtype} CUDA tensor of {numel} elements")


def image_downsample2(src, width, height, planes=1, precision="mixed", stream=None):
    """opt_image_downsample2: 2 x 2 block means; returns planes x H/2 x W/2."""
    _img_check(src, precision, planes * width * height, "src")
    dst = torch.empty((planes, height // 2, width // 2), dtype=src.dtype, device=src.device)
    _check(lib().opt_image_downsample2(_ptr(src), width, height, planes, PRECISIONS[precision], _ptr(dst),
                                       _stream_of(src, stream)), "opt_image_downsample2")
    return dst


def image_gradient(img, width, height, precision="mixed", stream=None):
    """opt_image_gradient: (dx, dy), each H x W."""
    _img_check(img, precision, width * height, "img")
    dx = torch.empty((height, width), dtype=img.dtype, device=img.device)
    dy = torch.empty_like(dx)
    _check(lib().opt_image_gradient(_ptr(img), width, height, PRECISIONS[precision], _ptr(dx), _ptr(dy),
                                    _stream_of(img, stream)), "opt_image_gradient")
    return dx, dy


def field_upsample(src, src_width, src_height, planes, scale, dst_width, dst_height, precision="mixed",
                   stream=None):
    """opt_field_upsample: planes x dst_height x dst_width."""
    _img_check(src, precision, planes * src_width * src_height, "src")
    sc = (ctypes.c_double * planes)(*[float(v) for v in scale])
    dst = torch.empty((planes, dst_height, dst_width), dtype=src.dtype, device=src.device)
    _check(lib().opt_field_upsample(_ptr(src), src_width, src_height, planes, sc, PRECISIONS[precision], _ptr(dst),
                                    dst_width, dst_height, _stream_of(src, stream)), "opt_field_upsample")
    return dst


def flow_pyramid_workspace_size(width, height, levels, precision="mixed"):
    b = ctypes.c_size_t(0)
    _check(lib().opt_flow_pyramid_workspace_size(width, height, levels, PRECISIONS[precision], ctypes.byref(b)),
           "opt_flow_pyramid_workspace_size")
    return b.value


def solve_flow_pyramid(I, I_hat, x, levels, w_fit, w_reg, precision="mixed", solve_params=None, stream=None,
                       workspace_bytes=None, report=True, **kw):
    """opt_solve_flow_pyramid on frames I, I_hat (H x W); x (2 x H x W) receives
    the flow.  Returns the per-level reports (level 0 = finest first), or None
    with report=False."""
    H, W = I.shape[-2], I.shape[-1]
    _img_check(I, precision, W * H, "I")
    _img_check(I_hat, precision, W * H, "I_hat")
    _img_check(x, precision, 2 * W * H, "x")
    nbytes = flow_pyramid_workspace_size(W, H, levels, precision) if workspace_bytes is None else workspace_bytes
    ws = torch.empty(max(int(nbytes), 1), dtype=torch.uint8, device=x.device)
    p = solve_params if solve_params is not None else default_params(**kw)
    traces = [(ctypes.c_double * (p.outer_iters + 1))() for _ in range(levels)]
    reps = (opt_solve_report * levels)()
    for k in range(levels):
        reps[k].cost_trace = ctypes.cast(traces[k], ctypes.POINTER(ctypes.c_double))
    code = lib().opt_solve_flow_pyramid(_ptr(I), _ptr(I_hat), W, H, levels, float(w_fit), float(w_reg),
                                        PRECISIONS[precision], ctypes.byref(p), _ptr(x), _ptr(ws), int(nbytes),
                                        _stream_of(x, stream), reps if report else None)
    _check(code, "opt_solve_flow_pyramid")
    if not report:
        return None
    return [dict(cost_initial=r.cost_initial, cost_final=r.cost_final, outer_done=r.outer_done,
                 steps_accepted=r.steps_accepted, cost_trace=list(t)) for r, t in zip(reps, traces)]


def workspace_size(energy, arrays, params=(), precision="mixed", width=0, height=0, n_vertices=0,
                   edges=None, depth=0):
    d, _, _ = make_desc(energy, arrays, params, precision, width, height, n_vertices, edges, depth)
    nbytes = ctypes.c_size_t(0)
    _check(lib().opt_workspace_size(ctypes.byref(d), ctypes.byref(nbytes)), "opt_workspace_size")
    return nbytes.value


class Server:
    """Continuous-batching server (opt_server_* in include/opt.h).

    ``arena_bytes`` of device memory are allocated here as one torch tensor and
    handed to the library: it is the memory budget of the requests held at once.
    ``tuning="auto"`` registers the committed tuning table in its served form
    (each entry's fastest launch shape with strips of at least four rows).
    """

    def __init__(self, arena_bytes, max_slots=64, device="cuda", stream=None, tuning="auto"):
        self.stream = stream if stream is not None else torch.cuda.current_stream(device)
        self.arena = torch.empty(int(arena_bytes), dtype=torch.uint8, device=device)
        h = ctypes.c_void_p(0)
        _check(lib().opt_server_create(_ptr(self.arena), self.arena.numel(), int(max_slots),
                                      ctypes.c_void_p(self.stream.cuda_stream), ctypes.byref(h)),
               "opt_server_create")
        self.handle = h
        self._lib = lib()
        self._held = {}  # ticket -> (desc, tensors, outer_iters), kept alive until collected
        if tuning == "auto":
            from . import tune
            tune.apply(self, tune.load())

    @staticmethod
    def reserved_bytes(max_slots):
        b = ctypes.c_size_t(0)
        _check(lib().opt_server_reserved_bytes(int(max_slots), ctypes.byref(b)), "opt_server_reserved_bytes")
        return b.value

    def __del__(self):
        # at interpreter exit the module globals may already be gone; the
        # library handle kept on the instance still works
        h = getattr(self, "handle", None)
        L = getattr(self, "_lib", None)
        if h is not None and h.value and L is not None:
            L.opt_server_destroy(h)
            self.handle = None

    def submit(self, energy, arrays, x, params=(), precision="mixed", width=0, height=0,
               n_vertices=0, edges=None, solve_params=None, depth=0, **kw):
        """Admit a request solving x in place; returns its ticket, or None when
        the server is full (OPT_EAGAIN)."""
        n_sites = n_vertices if n_vertices else width * height * (depth if depth else 1)
        check_request(energy, list(arrays), x, precision, n_sites, bool(n_vertices))
        d, arrays, edges = make_desc(energy, arrays, params, precision, width, height, n_vertices, edges, depth)
        sp = solve_params if solve_params is not None else default_params(**kw)
        t = ctypes.c_int64(-1)
        code = lib().opt_server_submit(self.handle, ctypes.byref(d), _ptr(x), ctypes.byref(sp),
                                       ctypes.byref(t))
        if code == OPT_EAGAIN:
            return None
        _check(code, "opt_server_submit")
        self._held[t.value] = (d, arrays, edges, x, sp.outer_iters)
        return t.value

    def step(self):
        _check(lib().opt_server_step(self.handle), "opt_server_step")

    def wait(self):
        _check(lib().opt_server_wait(self.handle), "opt_server_wait")

    def set_fill_budget(self, budget):
        _check(lib().opt_server_set_fill_budget(self.handle, float(budget)), "opt_server_set_fill_budget")

    def poll(self, ticket):
        """None while the request runs; its report (a dict) once it has left."""
        done = ctypes.c_int32(0)
        K = self._held[ticket][4] if ticket in self._held else 0
        trace = (ctypes.c_double * (K + 1))()
        rep = opt_solve_report()
        rep.cost_trace = ctypes.cast(trace, ctypes.POINTER(ctypes.c_double))
        code = lib().opt_server_poll(self.handle, int(ticket), ctypes.byref(done), ctypes.byref(rep))
        if code not in (OPT_OK, OPT_ENUMERIC):
            _check(code, "opt_server_poll")
        if not done.value:
            return None
        self._held.pop(ticket, None)
        return dict(cost_initial=rep.cost_initial, cost_final=rep.cost_final,
                    outer_done=rep.outer_done, steps_accepted=rep.steps_accepted,
                    cost_trace=list(trace), code=code)

    def cancel(self, ticket):
        _check(lib().opt_server_cancel(self.handle, int(ticket)), "opt_server_cancel")
        self._held.pop(ticket, None)

    def add_tuning(self, energy, precision, min_sites, max_sites, strip_rows=0, waves_per_simd=0,
                   large_grid_form=0):
        t = opt_tuning()
        t.strip_rows = int(strip_rows)
        t.waves_per_simd = int(waves_per_simd)
        t.large_grid_form = int(large_grid_form)
        _check(lib().opt_server_add_tuning(self.handle, ENERGIES[energy], PRECISIONS[precision],
                                           int(min_sites), int(max_sites), ctypes.byref(t)),
               "opt_server_add_tuning")

    def info(self):
        """(requests held, free arena bytes)."""
        a = ctypes.c_int32(0)
        f = ctypes.c_size_t(0)
        _check(lib().opt_server_info(self.handle, ctypes.byref(a), ctypes.byref(f)), "opt_server_info")
        return a.value, f.value
