"""Thin ctypes binding of libraygraph.so (include/raygraph.h).

Only argument marshalling lives here: graph construction, differentiation,
code generation and every step of the ray integration run in the C++
library and its gfx950 kernels.  PyTorch provides device memory and the
stream.  If the library is missing, importing this module raises.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Dict, List, Optional, Sequence

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libraygraph.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is missing: run `python -m paper_2508_15967_amd.build`")

# The library must share the process's HIP runtime with the caller that owns
# the device memory and streams (PyTorch here).  PyTorch ships its own
# libamdhip64; loading it first lets the dynamic loader satisfy this
# library's dependency with that same runtime instead of a second copy.
try:
    import torch  # noqa: F401
except ImportError:  # pragma: no cover - host-only use without torch
    pass

_lib = C.CDLL(LIB_PATH)


def _hip_runtimes():
    paths = set()
    with open("/proc/self/maps") as f:
        for line in f:
            path = line.split()[-1] if len(line.split()) >= 6 else ""
            if os.path.basename(path).startswith("libamdhip64.so"):
                paths.add(os.path.realpath(path))
    return sorted(paths)


if len(_hip_runtimes()) > 1:
    raise ImportError("two HIP runtimes are loaded in this process (%s); import torch before "
                      "any other HIP library so that one runtime serves both" % _hip_runtimes())

# status codes and enums (raygraph.h)
RG_OK, RG_EINVAL, RG_ENOMEM, RG_ECOMPILE, RG_EHIP, RG_EUNSUPPORTED, RG_ESTATE = 0, -1, -2, -3, -4, -5, -6
RG_X, RG_K, RG_OMEGA, RG_T = range(4)
RG_NEG, RG_EXP, RG_LOG, RG_SQRT, RG_SIN, RG_COS = range(6)
RG_ADD, RG_SUB, RG_MUL, RG_DIV = range(4)
(OP_CONST, OP_VAR, OP_PARAM, OP_ADD, OP_SUB, OP_MUL, OP_DIV, OP_NEG, OP_EXP, OP_LOG, OP_SQRT,
 OP_SIN, OP_COS, OP_POWI, OP_SPLINE) = range(15)
RK4, DOPRI54 = 0, 1
PERSISTENT, PLAIN = 0, 1
FP64, FP32 = 0, 1
RAY_OK, RAY_EXITED_BOX, RAY_BUDGET, RAY_NONFINITE, RAY_STEP_UNDERFLOW = range(5)

SYMBOLS = [
    "rg_create_graph", "rg_destroy_graph", "rg_node_var", "rg_node_const", "rg_node_param",
    "rg_node_elem", "rg_node_unary", "rg_node_binary", "rg_node_powi", "rg_node_bspline2",
    "rg_df", "rg_node_get", "rg_graph_size", "rg_eval", "rg_node_to_string", "rg_compile",
    "rg_destroy_program", "rg_program_info_get", "rg_program_source", "rg_program_functions",
    "rg_trace_rays", "rg_trace_rays_adjoint", "rg_eval_rays", "rg_last_launch", "rg_last_error",
    "rg_solve_k", "rg_workspace_size", "rg_adjoint_workspace_size", "rg_program_load",
    "rg_trace_rays_noalloc", "rg_trace_stats",
]


class RayGraphError(RuntimeError):
    def __init__(self, status: int, where: str):
        msg = _lib.rg_last_error().decode(errors="replace")
        super().__init__(f"{where} failed with status {status}: {msg}")
        self.status = status


class _CompileOpts(C.Structure):
    _fields_ = [("struct_size", C.c_uint32), ("want_adjoint", C.c_int32),
                ("compile_only", C.c_int32), ("opt_level", C.c_int32), ("arch", C.c_char_p),
                ("fp32", C.c_int32), ("deterministic", C.c_int32)]


class _ProgramInfo(C.Structure):
    _fields_ = [("struct_size", C.c_uint32), ("dim", C.c_uint32), ("n_params", C.c_uint32),
                ("n_grad_slots", C.c_uint32), ("n_nodes_rhs", C.c_uint32),
                ("n_nodes_vjp", C.c_uint32),
                ("rhs_flops_alg", C.c_double), ("rhs_flops_issued", C.c_double),
                ("rk4_step_flops_alg", C.c_double), ("rk4_step_flops_issued", C.c_double),
                ("dopri_attempt_flops_alg", C.c_double), ("dopri_attempt_flops_issued", C.c_double),
                ("vjp_flops_alg", C.c_double), ("vjp_flops_issued", C.c_double),
                ("adj_step_flops_alg", C.c_double), ("adj_step_flops_issued", C.c_double),
                ("source_hash", C.c_uint64), ("compile_ms", C.c_double),
                ("rhs_flops_ray_invariant", C.c_double), ("vjp_flops_ray_invariant", C.c_double)]


class _NodeDesc(C.Structure):
    _fields_ = [("op", C.c_int32), ("aux", C.c_int32), ("a", C.c_uint32), ("b", C.c_uint32),
                ("value", C.c_double)]


class TraceDesc(C.Structure):
    _fields_ = [("struct_size", C.c_uint32), ("n_rays", C.c_uint32),
                ("x0", C.c_void_p), ("k0", C.c_void_p), ("t0", C.c_void_p), ("omega", C.c_void_p),
                ("params", C.c_void_p),
                ("integrator", C.c_int32), ("n_steps", C.c_int32), ("dt", C.c_double),
                ("h0", C.c_double), ("rtol", C.c_double), ("atol", C.c_double), ("hmin", C.c_double),
                ("t_end", C.c_double), ("budget", C.c_void_p), ("max_steps", C.c_int32),
                ("has_box", C.c_int32), ("box_lo", C.c_double * 3), ("box_hi", C.c_double * 3),
                ("store_every", C.c_int32), ("traj", C.c_void_p), ("traj_D", C.c_void_p),
                ("x_out", C.c_void_p), ("k_out", C.c_void_p), ("t_out", C.c_void_p),
                ("status_out", C.c_void_p), ("steps_out", C.c_void_p),
                ("checkpoint_every", C.c_int32), ("checkpoints", C.c_void_p),
                ("mode", C.c_int32), ("use_hipgraph", C.c_int32), ("block", C.c_int32),
                ("rays_per_lane", C.c_int32), ("compact_interval", C.c_int32),
                ("attempts_out", C.c_void_p), ("precision", C.c_int32),
                ("workspace", C.c_void_p), ("workspace_bytes", C.c_size_t),
                ("min_waves_per_simd", C.c_int32)]


class AdjointDesc(C.Structure):
    _fields_ = [("struct_size", C.c_uint32), ("fwd", C.POINTER(TraceDesc)),
                ("dL_dx_end", C.c_void_p), ("dL_dk_end", C.c_void_p), ("dL_dx0", C.c_void_p),
                ("dL_dk0", C.c_void_p), ("dL_dparams", C.c_void_p),
                ("workspace", C.c_void_p), ("workspace_bytes", C.c_size_t)]


class SolveDesc(C.Structure):
    _fields_ = [("struct_size", C.c_uint32), ("n_rays", C.c_uint32), ("x", C.c_void_p),
                ("k", C.c_void_p), ("omega", C.c_void_p), ("t", C.c_void_p), ("params", C.c_void_p),
                ("component", C.c_int32), ("max_iter", C.c_int32), ("tol", C.c_double),
                ("D_out", C.c_void_p), ("iters_out", C.c_void_p), ("max_abs_D", C.c_void_p)]


class LaunchInfo(C.Structure):
    _fields_ = [("struct_size", C.c_uint32), ("block", C.c_int32), ("rays_per_lane", C.c_int32),
                ("compact_interval", C.c_int32), ("grid", C.c_int32), ("tuned", C.c_int32),
                ("min_waves_per_simd", C.c_int32), ("last_kernel_ms", C.c_double)]


_lib.rg_last_error.restype = C.c_char_p
for _name in SYMBOLS:
    if _name != "rg_last_error":
        getattr(_lib, _name).restype = C.c_int32


def _chk(status: int, where: str):
    if status != RG_OK:
        raise RayGraphError(status, where)


def exported_symbols() -> List[str]:
    """Names of SYMBOLS the loaded library exports."""
    out = []
    for s in SYMBOLS:
        try:
            getattr(_lib, s)
            out.append(s)
        except AttributeError:
            pass
    return out


# --------------------------------------------------------------------------
# graph

class Node:
    """A node of a Graph; arithmetic operators build new (reduced) nodes."""
    __slots__ = ("g", "id")

    def __init__(self, g: "Graph", nid: int):
        self.g, self.id = g, int(nid)

    def _lift(self, v) -> "Node":
        return v if isinstance(v, Node) else self.g.const(float(v))

    def _bin(self, op, other, rev=False):
        o = self._lift(other)
        a, b = (o, self) if rev else (self, o)
        out = C.c_uint32()
        _chk(_lib.rg_node_binary(self.g.h, op, a.id, b.id, C.byref(out)), "rg_node_binary")
        return Node(self.g, out.value)

    def __add__(self, o): return self._bin(RG_ADD, o)
    def __radd__(self, o): return self._bin(RG_ADD, o, True)
    def __sub__(self, o): return self._bin(RG_SUB, o)
    def __rsub__(self, o): return self._bin(RG_SUB, o, True)
    def __mul__(self, o): return self._bin(RG_MUL, o)
    def __rmul__(self, o): return self._bin(RG_MUL, o, True)
    def __truediv__(self, o): return self._bin(RG_DIV, o)
    def __rtruediv__(self, o): return self._bin(RG_DIV, o, True)

    def __neg__(self): return self.g.unary(RG_NEG, self)

    def __pow__(self, n):
        if int(n) != n:
            raise ValueError("only integer powers")
        out = C.c_uint32()
        _chk(_lib.rg_node_powi(self.g.h, self.id, int(n), C.byref(out)), "rg_node_powi")
        return Node(self.g, out.value)

    def exp(self): return self.g.unary(RG_EXP, self)
    def log(self): return self.g.unary(RG_LOG, self)
    def sqrt(self): return self.g.unary(RG_SQRT, self)
    def sin(self): return self.g.unary(RG_SIN, self)
    def cos(self): return self.g.unary(RG_COS, self)

    def df(self, wrt: "Node") -> "Node":
        return self.g.df(self, wrt)

    def desc(self) -> Dict:
        d = _NodeDesc()
        _chk(_lib.rg_node_get(self.g.h, self.id, C.byref(d)), "rg_node_get")
        return {"op": d.op, "aux": d.aux, "a": d.a, "b": d.b, "value": d.value}

    def is_const(self, v: Optional[float] = None) -> bool:
        d = self.desc()
        return d["op"] == OP_CONST and (v is None or d["value"] == v)

    def __repr__(self):
        return self.g.to_string(self)

    def __eq__(self, other):  # identity of hash-consed nodes
        return isinstance(other, Node) and other.g is self.g and other.id == self.id

    def __hash__(self):
        return hash((id(self.g), self.id))


class Graph:
    """Expression graph over x[dim], k[dim], omega and t (rg_create_graph)."""

    def __init__(self, dim: int):
        h = C.c_void_p()
        _chk(_lib.rg_create_graph(C.c_uint32(dim), C.byref(h)), "rg_create_graph")
        self.h = h
        self.dim = dim
        self.param_lens: List[int] = []
        self.param_names: List[str] = []

    def __del__(self):
        # module globals may already be cleared at interpreter exit
        if getattr(self, "h", None) and _lib is not None:
            _lib.rg_destroy_graph(self.h)
            self.h = None

    def _var(self, which, i=0):
        out = C.c_uint32()
        _chk(_lib.rg_node_var(self.h, which, C.c_uint32(i), C.byref(out)), "rg_node_var")
        return Node(self, out.value)

    def x(self, i: int) -> Node: return self._var(RG_X, i)
    def k(self, i: int) -> Node: return self._var(RG_K, i)

    @property
    def omega(self) -> Node: return self._var(RG_OMEGA)

    @property
    def t(self) -> Node: return self._var(RG_T)

    def const(self, v: float) -> Node:
        out = C.c_uint32()
        _chk(_lib.rg_node_const(self.h, C.c_double(v), C.byref(out)), "rg_node_const")
        return Node(self, out.value)

    def param(self, name: str, length: int) -> int:
        out = C.c_uint32()
        _chk(_lib.rg_node_param(self.h, name.encode(), C.c_uint32(length), C.byref(out)), "rg_node_param")
        self.param_lens.append(int(length))
        self.param_names.append(name)
        return out.value

    def elem(self, param: int, idx: int) -> Node:
        out = C.c_uint32()
        _chk(_lib.rg_node_elem(self.h, C.c_uint32(param), C.c_uint32(idx), C.byref(out)), "rg_node_elem")
        return Node(self, out.value)

    def unary(self, op: int, a: Node) -> Node:
        out = C.c_uint32()
        _chk(_lib.rg_node_unary(self.h, op, a.id, C.byref(out)), "rg_node_unary")
        return Node(self, out.value)

    def bspline2(self, param: int, nx: int, ny: int, lo, hi, u: Node, v: Node) -> Node:
        out = C.c_uint32()
        lo_a = (C.c_double * 2)(*lo)
        hi_a = (C.c_double * 2)(*hi)
        _chk(_lib.rg_node_bspline2(self.h, C.c_uint32(param), C.c_uint32(nx), C.c_uint32(ny), lo_a,
                                   hi_a, u.id, v.id, C.byref(out)), "rg_node_bspline2")
        return Node(self, out.value)

    def df(self, f: Node, wrt: Node) -> Node:
        out = C.c_uint32()
        _chk(_lib.rg_df(self.h, f.id, wrt.id, C.byref(out)), "rg_df")
        return Node(self, out.value)

    def size(self) -> int:
        n = C.c_uint32()
        _chk(_lib.rg_graph_size(self.h, C.byref(n)), "rg_graph_size")
        return n.value

    def eval(self, f: Node, x, k, omega=1.0, t=0.0, params: Sequence[np.ndarray] = ()) -> float:
        xa = (C.c_double * self.dim)(*[float(v) for v in x])
        ka = (C.c_double * self.dim)(*[float(v) for v in k])
        arrs = [np.ascontiguousarray(p, dtype=np.float64) for p in params]
        pp = (C.c_void_p * max(1, len(arrs)))(*[a.ctypes.data for a in arrs]) if arrs else None
        out = C.c_double()
        _chk(_lib.rg_eval(self.h, f.id, xa, ka, C.c_double(omega), C.c_double(t), pp, C.byref(out)),
             "rg_eval")
        return out.value

    def to_string(self, n: Node) -> str:
        need = C.c_size_t()
        _chk(_lib.rg_node_to_string(self.h, n.id, None, 0, C.byref(need)), "rg_node_to_string")
        buf = C.create_string_buffer(need.value)
        _chk(_lib.rg_node_to_string(self.h, n.id, buf, need.value, None), "rg_node_to_string")
        return buf.value.decode()

    def compile(self, D: Node, want_adjoint: bool = False, compile_only: bool = False,
                opt_level: int = 0, fp32: bool = False, deterministic: bool = False) -> "Program":
        o = _CompileOpts(C.sizeof(_CompileOpts), int(want_adjoint), int(compile_only), opt_level, None,
                         int(fp32), int(deterministic))
        h = C.c_void_p()
        _chk(_lib.rg_compile(self.h, D.id, C.byref(o), C.byref(h)), "rg_compile")
        return Program(h, self.dim, list(self.param_lens), list(self.param_names))


# --------------------------------------------------------------------------
# program

def _dptr(t) -> Optional[int]:
    return None if t is None else int(t.data_ptr())


def _stream_handle(stream) -> int:
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return int(s.cuda_stream)


def _check_tensor(t, name, dtype=None):
    import torch
    if t is None:
        return
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a GPU tensor")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if dtype is not None and t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}")


class Program:
    """A compiled ray program (rg_compile)."""

    def __init__(self, h, dim, param_lens, param_names):
        self.h = h
        self.dim = dim
        self.param_lens = param_lens
        self.param_names = param_names

    def __del__(self):
        # module globals may already be cleared at interpreter exit
        if getattr(self, "h", None) and _lib is not None:
            _lib.rg_destroy_program(self.h)
            self.h = None

    def info(self) -> Dict:
        i = _ProgramInfo()
        i.struct_size = C.sizeof(_ProgramInfo)
        _chk(_lib.rg_program_info_get(self.h, C.byref(i)), "rg_program_info_get")
        return {f: getattr(i, f) for f, _ in _ProgramInfo._fields_ if f != "struct_size"}

    def source(self) -> str:
        p = C.c_char_p()
        _chk(_lib.rg_program_source(self.h, C.byref(p)), "rg_program_source")
        return p.value.decode()

    def functions(self) -> str:
        p = C.c_char_p()
        _chk(_lib.rg_program_functions(self.h, C.byref(p)), "rg_program_functions")
        return p.value.decode()

    def last_launch(self) -> Dict:
        li = LaunchInfo()
        _chk(_lib.rg_last_launch(self.h, C.byref(li)), "rg_last_launch")
        return {f: getattr(li, f) for f, _ in LaunchInfo._fields_ if f != "struct_size"}

    # -- descriptors -------------------------------------------------------
    def make_desc(self, x0, k0, omega, params=(), *, integrator=RK4, dt=0.0, n_steps=0, h0=0.0,
                  rtol=0.0, atol=0.0, hmin=0.0, t_end=0.0, budget=None, max_steps=0, box=None,
                  t0=None, store_every=0, traj=None, traj_D=None, x_out=None, k_out=None,
                  t_out=None, status_out=None, steps_out=None, checkpoint_every=0,
                  checkpoints=None, mode=PERSISTENT, use_hipgraph=False, block=0,
                  rays_per_lane=0, compact_interval=0, attempts_out=None, precision=FP64,
                  workspace=None, min_waves_per_simd=0):
        import torch
        f64, i32 = torch.float64, torch.int32
        for t, nm, dt_ in ((x0, "x0", f64), (k0, "k0", f64), (omega, "omega", f64), (t0, "t0", f64),
                           (budget, "budget", i32), (traj, "traj", f64), (traj_D, "traj_D", f64),
                           (x_out, "x_out", f64), (k_out, "k_out", f64), (t_out, "t_out", f64),
                           (status_out, "status_out", i32), (steps_out, "steps_out", i32),
                           (checkpoints, "checkpoints", f64), (attempts_out, "attempts_out", i32)):
            _check_tensor(t, nm, dt_)
        if len(params) != len(self.param_lens):
            raise ValueError(f"expected {len(self.param_lens)} parameter arrays, got {len(params)}")
        for p in params:
            _check_tensor(p, "param", f64)
        d = TraceDesc()
        d.struct_size = C.sizeof(TraceDesc)
        # the descriptor holds every tensor it points to, so that a later
        # call on it (the adjoint reads x0, k0, omega, the parameters, the
        # checkpoints and the step counts) never sees freed memory
        d._refs = (x0, k0, omega, t0, budget, traj, traj_D, x_out, k_out, t_out, status_out, steps_out,
                   checkpoints, attempts_out, tuple(params))
        d.n_rays = int(x0.shape[-1])
        d.x0, d.k0, d.t0, d.omega = _dptr(x0), _dptr(k0), _dptr(t0), _dptr(omega)
        pp = (C.c_void_p * max(1, len(params)))(*[_dptr(p) for p in params])
        d._keep = pp  # the pointer array lives as long as the descriptor
        d.params = C.cast(pp, C.c_void_p).value if params else None
        d.integrator, d.n_steps, d.dt = integrator, int(n_steps), float(dt)
        d.h0, d.rtol, d.atol, d.hmin, d.t_end = float(h0), float(rtol), float(atol), float(hmin), float(t_end)
        d.budget, d.max_steps = _dptr(budget), int(max_steps)
        if box is not None:
            lo, hi = box
            d.has_box = 1
            d.box_lo[:] = list(lo) + [0.0] * (3 - len(lo))
            d.box_hi[:] = list(hi) + [0.0] * (3 - len(hi))
        d.store_every, d.traj, d.traj_D = int(store_every), _dptr(traj), _dptr(traj_D)
        d.x_out, d.k_out, d.t_out = _dptr(x_out), _dptr(k_out), _dptr(t_out)
        d.status_out, d.steps_out = _dptr(status_out), _dptr(steps_out)
        d.checkpoint_every, d.checkpoints = int(checkpoint_every), _dptr(checkpoints)
        d.mode, d.use_hipgraph = int(mode), int(bool(use_hipgraph))
        d.block, d.rays_per_lane, d.compact_interval = int(block), int(rays_per_lane), int(compact_interval)
        d.attempts_out = _dptr(attempts_out)
        d.precision = int(precision)
        d.min_waves_per_simd = int(min_waves_per_simd)
        # per-call scratch: a torch allocation of the size the library asks for
        if d.n_rays > 0:
            need = self.workspace_size(d)
            if need > 0:
                if workspace is None:
                    workspace = torch.empty(need, dtype=torch.uint8, device=x0.device)
                _check_tensor(workspace, "workspace")
                d.workspace, d.workspace_bytes = _dptr(workspace), workspace.numel() * workspace.element_size()
                d._ws = workspace
        return d

    def workspace_size(self, d: TraceDesc) -> int:
        """Bytes of device workspace rg_trace_rays needs for d."""
        b = C.c_size_t()
        _chk(_lib.rg_workspace_size(self.h, C.byref(d), C.byref(b)), "rg_workspace_size")
        return int(b.value)

    def adjoint_workspace_size(self, a: "AdjointDesc") -> int:
        b = C.c_size_t()
        _chk(_lib.rg_adjoint_workspace_size(self.h, C.byref(a), C.byref(b)), "rg_adjoint_workspace_size")
        return int(b.value)

    def trace_stats(self, d: TraceDesc, stream=None) -> Dict:
        """Solver statistics of a finished trace (rg_trace_stats), on the host."""
        import torch
        dev = torch.device("cuda", torch.cuda.current_device())
        st = torch.empty(10, dtype=torch.int64, device=dev)
        _chk(_lib.rg_trace_stats(self.h, C.byref(d), C.c_void_p(_dptr(st)),
                                 C.c_void_p(_stream_handle(stream))), "rg_trace_stats")
        v = [int(x) for x in st.cpu().tolist()]
        return {"by_status": {s: v[s] for s in range(5)}, "other_status": v[5], "steps": v[6],
                "attempts": v[7], "rejected": v[7] - v[6] if v[7] else 0, "max_steps": v[8],
                "max_attempts": v[9]}

    def load(self):
        """Load the code object on the current device (rg_program_load)."""
        _chk(_lib.rg_program_load(self.h), "rg_program_load")

    def trace_desc_noalloc(self, d: TraceDesc, stream=None):
        """rg_trace_rays_noalloc: scratch from the library's static device
        array (d.workspace is ignored); launch parameters must be given."""
        _chk(_lib.rg_trace_rays_noalloc(self.h, C.byref(d), C.c_void_p(_stream_handle(stream))),
             "rg_trace_rays_noalloc")

    def trace_desc(self, d: TraceDesc, stream=None):
        _chk(_lib.rg_trace_rays(self.h, C.byref(d), C.c_void_p(_stream_handle(stream))), "rg_trace_rays")

    def adjoint_desc(self, fwd: TraceDesc, dL_dx_end, dL_dk_end=None, dL_dx0=None, dL_dk0=None,
                     dL_dparams=(), stream=None, workspace=None):
        """Adjoint of the trace described by fwd.  The workspace (a torch
        allocation of the size the library reports) is kept on fwd and reused
        by later calls that need no more."""
        import torch
        for t, nm in ((dL_dx_end, "dL_dx_end"), (dL_dk_end, "dL_dk_end"), (dL_dx0, "dL_dx0"),
                      (dL_dk0, "dL_dk0")):
            _check_tensor(t, nm)
        a = AdjointDesc()
        a.struct_size = C.sizeof(AdjointDesc)
        a.fwd = C.pointer(fwd)
        a.dL_dx_end, a.dL_dk_end = _dptr(dL_dx_end), _dptr(dL_dk_end)
        a.dL_dx0, a.dL_dk0 = _dptr(dL_dx0), _dptr(dL_dk0)
        gp = list(dL_dparams) + [None] * (len(self.param_lens) - len(dL_dparams))
        gpa = (C.c_void_p * max(1, len(gp)))(*[_dptr(g) for g in gp])
        a._keep = gpa
        a.dL_dparams = C.cast(gpa, C.c_void_p).value if gp else None
        if fwd.n_rays > 0:
            need = self.adjoint_workspace_size(a)
            if need > 0:
                if workspace is None:
                    workspace = getattr(fwd, "_adj_ws", None)
                    if workspace is None or workspace.numel() < need:
                        fwd._adj_ws = None
                        workspace = torch.empty(need, dtype=torch.uint8, device=dL_dx_end.device)
                        fwd._adj_ws = workspace
                _check_tensor(workspace, "workspace")
                a.workspace, a.workspace_bytes = _dptr(workspace), workspace.numel() * workspace.element_size()
        _chk(_lib.rg_trace_rays_adjoint(self.h, C.byref(a), C.c_void_p(_stream_handle(stream))),
             "rg_trace_rays_adjoint")

    # -- convenience -------------------------------------------------------
    def trace(self, x0, k0, omega, params=(), *, store=False, store_D=False, checkpoint_every=0,
              stream=None, **kw):
        """Allocate outputs with torch and trace.  Returns a dict of tensors."""
        import torch
        dev = x0.device
        n = int(x0.shape[-1])
        d, ny = self.dim, 2 * self.dim
        out = {"x": torch.empty((d, n), dtype=torch.float64, device=dev),
               "k": torch.empty((d, n), dtype=torch.float64, device=dev),
               "t": torch.empty(n, dtype=torch.float64, device=dev),
               "status": torch.empty(n, dtype=torch.int32, device=dev),
               "steps": torch.empty(n, dtype=torch.int32, device=dev)}
        if kw.get("integrator", RK4) == DOPRI54:
            out["attempts"] = torch.empty(n, dtype=torch.int32, device=dev)
        se = int(kw.pop("store_every", 0))
        if (store or store_D) and se > 0:
            ns = int(kw.get("n_steps", 0)) // se + 1
            if store:
                out["traj"] = torch.empty((ns, ny, n), dtype=torch.float64, device=dev)
            if store_D:
                out["traj_D"] = torch.empty((ns, n), dtype=torch.float64, device=dev)
        else:
            se = 0
        if checkpoint_every > 0:
            nc = (int(kw.get("n_steps", 0)) + checkpoint_every - 1) // checkpoint_every
            out["checkpoints"] = torch.empty((nc, ny + 1, n), dtype=torch.float64, device=dev)
        desc = self.make_desc(x0, k0, omega, params, store_every=se, traj=out.get("traj"),
                              traj_D=out.get("traj_D"), x_out=out["x"], k_out=out["k"],
                              t_out=out["t"], status_out=out["status"], steps_out=out["steps"],
                              checkpoint_every=checkpoint_every, checkpoints=out.get("checkpoints"),
                              attempts_out=out.get("attempts"), **kw)
        self.trace_desc(desc, stream)
        out["_desc"] = desc
        return out

    def solve_k(self, x, k, omega, params=(), component=0, tol=1e-15, max_iter=50, stream=None):
        """Newton solve of D = 0 for k[component] in place (rg_solve_k).
        Returns (iterations per ray, final D per ray, max |D| as a 1-element tensor)."""
        import torch
        for t, nm in ((x, "x"), (k, "k"), (omega, "omega")):
            _check_tensor(t, nm, torch.float64)
        for p in params:
            _check_tensor(p, "param", torch.float64)
        n = int(x.shape[-1])
        dev = x.device
        it = torch.empty(n, dtype=torch.int32, device=dev)
        D = torch.empty(n, dtype=torch.float64, device=dev)
        mx = torch.empty(1, dtype=torch.float64, device=dev)
        d = SolveDesc()
        d.struct_size = C.sizeof(SolveDesc)
        d.n_rays = n
        d.x, d.k, d.omega = _dptr(x), _dptr(k), _dptr(omega)
        pp = (C.c_void_p * max(1, len(params)))(*[_dptr(p) for p in params])
        d.params = C.cast(pp, C.c_void_p).value if params else None
        d.component, d.max_iter, d.tol = int(component), int(max_iter), float(tol)
        d.D_out, d.iters_out, d.max_abs_D = _dptr(D), _dptr(it), _dptr(mx)
        _chk(_lib.rg_solve_k(self.h, C.byref(d), C.c_void_p(_stream_handle(stream))), "rg_solve_k")
        return it, D, mx

    def eval(self, y, omega, params=(), t=None, stream=None):
        """Right-hand side f [2d][n] and D [n] at points y [2d][n] on the GPU."""
        import torch
        _check_tensor(y, "y", torch.float64)
        _check_tensor(omega, "omega", torch.float64)
        _check_tensor(t, "t", torch.float64)
        for p in params:
            _check_tensor(p, "param", torch.float64)
        n = int(y.shape[-1])
        f = torch.empty_like(y)
        D = torch.empty(n, dtype=torch.float64, device=y.device)
        pp = (C.c_void_p * max(1, len(params)))(*[_dptr(p) for p in params])
        _chk(_lib.rg_eval_rays(self.h, C.c_uint32(n), C.c_void_p(_dptr(y)), C.c_void_p(_dptr(omega)),
                               C.c_void_p(_dptr(t)) if t is not None else None,
                               pp if params else None, C.c_void_p(_dptr(f)), C.c_void_p(_dptr(D)),
                               C.c_void_p(_stream_handle(stream))), "rg_eval_rays")
        return f, D
