"""ctypes binding of libswf.so (argument marshalling only).

Every computation happens in the HIP library; this module converts the
problem description (``swf_workloads``) into the C structs of
``include/swf.h``, passes a torch-owned device workspace and torch's current
HIP stream, and converts results back to numpy.  Importing it raises if the
library has not been built: there is no fallback path.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libswf.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is missing: build it with paper_2512_16889_amd.build.build() "
                      "(the SWF solver has no non-HIP path)")

# torch is loaded first so that libswf.so binds to the HIP runtime torch
# already mapped (same soname): one runtime in the process, so torch's device
# memory and streams are valid handles inside the library.
import torch  # noqa: E402,F401

_lib = C.CDLL(LIB_PATH)

SWF_OK, SWF_E_ARG, SWF_E_NOMEM, SWF_E_HIP, SWF_E_ORDER, SWF_E_UNSUPPORTED, SWF_E_NONFINITE = range(7)
SWF_FP64, SWF_MIXED = 0, 1
SWF_RK4, SWF_DP5, SWF_IPRK4 = 0, 1, 2
STEPPERS = {"rk4": SWF_RK4, "dp5": SWF_DP5, "iprk4": SWF_IPRK4}
AMP_PAIR1, AMP_PAIR2, AMP_BW, AMP_BW_PARTIAL = 0, 1, 2, 3
P_MARGINAL_E, P_MARGINAL_POS, P_PAIR, P_BW = 0, 1, 2, 3
STAT_ROW, STAT_COLY, STAT_COLZ, STAT_BW, STAT_OTHER = range(5)


class Profile(C.Structure):
    _fields_ = [("type", C.c_int), ("c", C.c_double), ("w", C.c_double), ("k", C.c_double), ("phi", C.c_double)]


class Term(C.Structure):
    _fields_ = [("mu", C.c_int), ("amp", C.c_double), ("ft", Profile), ("fx", Profile * 3)]


class Grid(C.Structure):
    _fields_ = [("dim", C.c_int), ("n", C.c_int * 3), ("L", C.c_double * 3), ("absorb_cells", C.c_int),
                ("absorb_strength", C.c_double)]


class Window(C.Structure):
    _fields_ = [("t_in", C.c_double), ("t_out", C.c_double), ("dt", C.c_double)]


class Solve(C.Structure):
    _fields_ = [("kind", C.c_int), ("spin", C.c_int), ("p", C.c_double * 3), ("grid", C.c_int),
                ("field", C.c_int)]


class Vertex(C.Structure):
    _fields_ = [("u_solve", C.c_int), ("v_solve", C.c_int), ("k", C.c_double * 3), ("eps", C.c_double * 3),
                ("n_modes", C.c_int), ("modes", C.POINTER(C.c_double))]


class Options(C.Structure):
    _fields_ = [("prec", C.c_int), ("stream", C.c_void_p), ("workspace", C.c_void_p),
                ("workspace_bytes", C.c_size_t), ("use_graph", C.c_int), ("batched", C.c_int),
                ("profile", C.c_int), ("tune", C.c_int), ("tune_cache", C.c_char_p), ("chunk", C.c_int),
                ("force_variant", C.c_int), ("persistent", C.c_int), ("bw_partial", C.c_int),
                ("check_every", C.c_int), ("stepper", C.c_int), ("graph_steps", C.c_int)]


_P = C.POINTER
_lib.swf_workspace_size.argtypes = [_P(Grid), C.c_int, _P(Term), _P(C.c_int), C.c_int, _P(Solve), C.c_int,
                                    _P(Vertex), C.c_int, _P(Window), _P(Options), _P(C.c_size_t)]
_lib.swf_init.argtypes = [_P(Grid), C.c_int, _P(Term), _P(C.c_int), C.c_int, _P(Solve), C.c_int,
                          _P(Vertex), C.c_int, _P(Window), _P(Options), _P(C.c_void_p)]
_lib.swf_step.argtypes = [C.c_void_p, C.c_int, _P(C.c_int)]
_lib.swf_sync.argtypes = [C.c_void_p]
_lib.swf_reset.argtypes = [C.c_void_p]
_lib.swf_amplitude.argtypes = [C.c_void_p, C.c_int, C.c_int, C.c_int, _P(C.c_double)]
_lib.swf_probability.argtypes = [C.c_void_p, C.c_int, C.c_int, C.c_int, _P(C.c_double)]
_lib.swf_diagnostics.argtypes = [C.c_void_p, C.c_int, _P(C.c_double)]
_lib.swf_get_psi.argtypes = [C.c_void_p, C.c_int, _P(C.c_double)]
_lib.swf_set_psi.argtypes = [C.c_void_p, C.c_int, _P(C.c_double), C.c_int]
_lib.swf_get_bw_state.argtypes = [C.c_void_p, C.c_int, _P(C.c_double)]
_lib.swf_set_bw_state.argtypes = [C.c_void_p, C.c_int, _P(C.c_double)]
_lib.swf_apply_op.argtypes = [C.c_void_p, C.c_int, C.c_int, C.c_double, _P(C.c_double), _P(C.c_double)]
_lib.swf_kernel_stats.argtypes = [C.c_void_p, C.c_int, _P(C.c_longlong), _P(C.c_double), _P(C.c_double)]
_lib.swf_reset_stats.argtypes = [C.c_void_p]
_lib.swf_steps.argtypes = [C.c_void_p, _P(C.c_int), _P(C.c_int)]
_lib.swf_supported_n.argtypes = [C.c_int]
_lib.swf_pair_matrix.argtypes = [C.c_void_p, C.c_int, _P(C.c_int), C.c_int, _P(C.c_int), C.c_int, _P(C.c_double)]
_lib.swf_pair_matrix.restype = C.c_int
_lib.swf_pair_matrix_noalloc.argtypes = [C.c_void_p, C.c_int, _P(C.c_int), C.c_int, _P(C.c_int), C.c_int,
                                         _P(C.c_double)]
_lib.swf_pair_matrix_noalloc.restype = C.c_int
_lib.swf_noalloc_scratch_bytes.argtypes = []
_lib.swf_noalloc_scratch_bytes.restype = C.c_size_t
_lib.swf_tune_report.argtypes = [C.c_void_p]
_lib.swf_tune_report.restype = C.c_char_p
_lib.swf_last_error.argtypes = [C.c_void_p]
_lib.swf_last_error.restype = C.c_char_p
_lib.swf_free.argtypes = [C.c_void_p]
_lib.swf_free.restype = None

EXPORTED = ["swf_workspace_size", "swf_init", "swf_step", "swf_reset", "swf_sync", "swf_amplitude", "swf_probability",
            "swf_diagnostics", "swf_get_psi", "swf_set_psi", "swf_get_bw_state", "swf_set_bw_state",
            "swf_apply_op", "swf_kernel_stats", "swf_reset_stats", "swf_supported_n", "swf_steps",
            "swf_tune_report", "swf_last_error", "swf_free", "swf_pair_matrix", "swf_pair_matrix_noalloc",
            "swf_noalloc_scratch_bytes"]


class SwfError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"swf status {code}: {msg}")
        self.code = code


def noalloc_scratch_bytes() -> int:
    return int(_lib.swf_noalloc_scratch_bytes())


def supported_n(n: int) -> bool:
    return bool(_lib.swf_supported_n(int(n)))


def _profile(p):
    return Profile(int(p.type), float(p.c), float(p.w), float(p.k), float(p.phi))


def marshal(problem):
    """C arrays for the problem description."""
    grids = (Grid * len(problem.grids))()
    for i, g in enumerate(problem.grids):
        grids[i].dim = int(g.dim)
        for j in range(3):
            grids[i].n[j] = int(g.n[j])
            grids[i].L[j] = float(g.L[j])
        grids[i].absorb_cells = int(g.absorb_cells)
        grids[i].absorb_strength = float(g.absorb_strength)
    flat, first = [], [0]
    for f in problem.fields:
        flat.extend(f)
        first.append(len(flat))
    terms = (Term * max(1, len(flat)))()
    for i, t in enumerate(flat):
        terms[i].mu = int(t.mu)
        terms[i].amp = float(t.amp)
        terms[i].ft = _profile(t.ft)
        for j in range(3):
            terms[i].fx[j] = _profile(t.fx[j])
    ffirst = (C.c_int * len(first))(*first)
    solves = (Solve * len(problem.solves))()
    for i, s in enumerate(problem.solves):
        solves[i].kind = int(s.kind)
        solves[i].spin = int(s.spin)
        for j in range(3):
            solves[i].p[j] = float(s.p[j])
        solves[i].grid = int(s.grid)
        solves[i].field = int(s.field)
    verts = (Vertex * max(1, len(problem.vertices)))()
    verts.mode_arrays = []      # kept alive with the vertex array
    for i, v in enumerate(problem.vertices):
        verts[i].u_solve = int(v.u_solve)
        verts[i].v_solve = int(v.v_solve)
        for j in range(3):
            verts[i].k[j] = float(v.k[j])
            verts[i].eps[j] = float(v.eps[j])
        modes = getattr(v, "modes", None) or []
        verts[i].n_modes = len(modes)
        if modes:
            flat = []
            for k, e, c in modes:
                c = complex(c)
                flat += [float(k[0]), float(k[1]), float(k[2]), float(e[0]), float(e[1]), float(e[2]), c.real, c.imag]
            arr = (C.c_double * len(flat))(*flat)
            verts.mode_arrays.append(arr)
            verts[i].modes = C.cast(arr, C.POINTER(C.c_double))
    win = Window(float(problem.window.t_in), float(problem.window.t_out), float(problem.window.dt))
    return grids, terms, ffirst, solves, verts, win


def workspace_size(problem, precision: str = "fp64", bw_partial: bool = False) -> int:
    """Device bytes swf_init needs for this problem (swf_workspace_size); allocates nothing."""
    grids, terms, ffirst, solves, verts, win = marshal(problem)
    opt = Options()
    opt.prec = SWF_FP64 if precision == "fp64" else SWF_MIXED
    opt.batched = 1
    opt.bw_partial = int(bw_partial)
    opt.stepper = STEPPERS[getattr(problem.window, "scheme", "rk4")]
    nbytes = C.c_size_t(0)
    code = _lib.swf_workspace_size(grids, len(problem.grids), terms, ffirst, len(problem.fields), solves,
                                   len(problem.solves), verts, len(problem.vertices), C.byref(win), C.byref(opt),
                                   C.byref(nbytes))
    if code != SWF_OK:
        raise SwfError(code, _lib.swf_last_error(None).decode())
    return int(nbytes.value)


class Context:
    """One swf_ctx: all solves of a problem, stepped together."""

    def __init__(self, problem, precision: str = "fp64", use_graph: bool = False, batched: bool = True,
                 profile: bool = False, device_workspace: bool = True, tune: bool = False,
                 tune_cache: str | None = None, chunk: int = 0, variant: int | None = None,
                 persistent: bool = True, bw_partial: bool = False, check_every: int = 0, graph_steps: int = 0):
        if not torch.cuda.is_available():
            raise RuntimeError("the SWF solver runs on the GPU only; no device is visible")
        self.problem = problem
        self._arrays = marshal(problem)
        grids, terms, ffirst, solves, verts, win = self._arrays
        self.opt = Options()
        self.opt.prec = SWF_FP64 if precision == "fp64" else SWF_MIXED
        self.opt.use_graph = int(use_graph)
        self.opt.batched = int(batched)
        self.opt.profile = int(profile)
        self.opt.tune = int(tune)
        self.opt.chunk = int(chunk)
        self.opt.force_variant = 0 if variant is None else int(variant) + 1
        self.opt.persistent = int(persistent)
        self.opt.bw_partial = int(bw_partial)
        self.opt.check_every = int(check_every)
        self.opt.graph_steps = int(graph_steps)
        self.opt.stepper = STEPPERS[getattr(problem.window, "scheme", "rk4")]
        self._tune_cache = tune_cache.encode() if tune_cache else None
        self.opt.tune_cache = self._tune_cache
        self.opt.stream = C.c_void_p(torch.cuda.current_stream().cuda_stream)
        nbytes = C.c_size_t(0)
        args = (grids, len(problem.grids), terms, ffirst, len(problem.fields), solves, len(problem.solves),
                verts, len(problem.vertices), C.byref(win))
        self._check(_lib.swf_workspace_size(*args, C.byref(self.opt), C.byref(nbytes)), None)
        self.workspace_bytes = int(nbytes.value)
        self._ws = None
        if device_workspace:
            self._ws = torch.empty(self.workspace_bytes + 256, dtype=torch.uint8, device="cuda")
            ptr = self._ws.data_ptr()
            ptr = (ptr + 255) & ~255
            self.opt.workspace = C.c_void_p(ptr)
            self.opt.workspace_bytes = self.workspace_bytes
        self._ctx = C.c_void_p()
        self._check(_lib.swf_init(*args, C.byref(self.opt), C.byref(self._ctx)), None)

    # ---------------------------------------------------------------- utils
    def _check(self, code, ctx="self"):
        if code != SWF_OK:
            c = self._ctx if (ctx == "self" and getattr(self, "_ctx", None)) else None
            raise SwfError(code, _lib.swf_last_error(c).decode())

    def close(self):
        if getattr(self, "_ctx", None):
            _lib.swf_free(self._ctx)
            self._ctx = None
        self._ws = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    # ---------------------------------------------------------------- stepping
    def step(self, n: int | None = None) -> int:
        left = C.c_int(0)
        if n is None:
            total, done = self.steps()
            n = total - done
        self._check(_lib.swf_step(self._ctx, int(n), C.byref(left)))
        return left.value

    def sync(self):
        self._check(_lib.swf_sync(self._ctx))

    def reset(self):
        self._check(_lib.swf_reset(self._ctx))

    def steps(self):
        t, d = C.c_int(0), C.c_int(0)
        self._check(_lib.swf_steps(self._ctx, C.byref(t), C.byref(d)))
        return t.value, d.value

    # ---------------------------------------------------------------- observables
    def amplitude(self, which: int, i: int, j: int) -> complex:
        out = (C.c_double * 2)()
        self._check(_lib.swf_amplitude(self._ctx, which, i, j, out))
        return complex(out[0], out[1])

    def probability(self, which: int, i: int, j: int = -1) -> float:
        out = C.c_double(0)
        self._check(_lib.swf_probability(self._ctx, which, i, j, C.byref(out)))
        return out.value

    def marginal(self, i: int) -> float:
        kind = self.problem.solves[i].kind
        return self.probability(P_MARGINAL_E if kind % 2 == 0 else P_MARGINAL_POS, i)

    def pair(self, i: int, j: int, form: int = 1) -> complex:
        return self.amplitude(AMP_PAIR1 if form == 1 else AMP_PAIR2, i, j)

    def bw(self, v: int, term: int = -1) -> complex:
        return self.amplitude(AMP_BW, v, term)

    def bw_partial(self, v: int, term: int = -1) -> complex:
        return self.amplitude(AMP_BW_PARTIAL, v, term)

    def diagnostics(self, i: int):
        out = (C.c_double * 4)()
        self._check(_lib.swf_diagnostics(self._ctx, i, out))
        return tuple(out)

    # ---------------------------------------------------------------- state I/O
    def _shape(self, i):
        g = self.problem.grids[self.problem.solves[i].grid]
        return [int(g.n[j]) for j in range(g.dim)]

    def _to_lib(self, arr, i):
        n = self._shape(i)
        a = np.asarray(arr, dtype=np.complex128).reshape([4] + n)
        a = np.transpose(a, [0] + list(range(len(n), 0, -1)))     # x fastest
        return np.ascontiguousarray(a).view(np.float64).reshape(-1)

    def _from_lib(self, flat, i):
        n = self._shape(i)
        a = flat.view(np.complex128).reshape([4] + n[::-1])
        return np.ascontiguousarray(np.transpose(a, [0] + list(range(len(n), 0, -1))))

    def get_psi(self, i: int) -> np.ndarray:
        n = self._shape(i)
        buf = np.empty(8 * int(np.prod(n)), dtype=np.float64)
        self._check(_lib.swf_get_psi(self._ctx, i, buf.ctypes.data_as(_P(C.c_double))))
        return self._from_lib(buf, i)

    def set_psi(self, i: int, psi, step_index: int):
        buf = self._to_lib(psi, i)
        self._check(_lib.swf_set_psi(self._ctx, i, buf.ctypes.data_as(_P(C.c_double)), int(step_index)))

    def get_bw_state(self, v: int) -> np.ndarray:
        out = np.empty(6, dtype=np.float64)
        self._check(_lib.swf_get_bw_state(self._ctx, v, out.ctypes.data_as(_P(C.c_double))))
        return out.view(np.complex128)

    def set_bw_state(self, v: int, m):
        buf = np.ascontiguousarray(np.asarray(m, dtype=np.complex128)).view(np.float64)
        self._check(_lib.swf_set_bw_state(self._ctx, v, buf.ctypes.data_as(_P(C.c_double))))

    def apply_op(self, op: int, i: int, psi, t: float = 0.0) -> np.ndarray:
        inp = self._to_lib(psi, i)
        out = np.empty_like(inp)
        self._check(_lib.swf_apply_op(self._ctx, op, i, float(t), inp.ctypes.data_as(_P(C.c_double)),
                                      out.ctypes.data_as(_P(C.c_double))))
        return self._from_lib(out, i)

    # ---------------------------------------------------------------- profiling
    def pair_matrix(self, u_solves, v_solves, form: int = 1, noalloc: bool = False):
        """Omega(u_solves[m], v_solves[n]) for every pair, as an nu x nv complex array
        (noalloc: through swf_pair_matrix_noalloc, scratch in the static device array)."""
        us = (C.c_int * len(u_solves))(*[int(i) for i in u_solves])
        vs = (C.c_int * len(v_solves))(*[int(i) for i in v_solves])
        out = np.zeros(2 * len(u_solves) * len(v_solves), dtype=np.float64)
        fn = _lib.swf_pair_matrix_noalloc if noalloc else _lib.swf_pair_matrix
        self._check(fn(self._ctx, int(form), us, len(u_solves), vs, len(v_solves), out.ctypes.data_as(_P(C.c_double))))
        return (out[0::2] + 1j * out[1::2]).reshape(len(u_solves), len(v_solves))

    def kernel_stats(self, kind: int):
        n, ms, by = C.c_longlong(0), C.c_double(0), C.c_double(0)
        self._check(_lib.swf_kernel_stats(self._ctx, kind, C.byref(n), C.byref(ms), C.byref(by)))
        return n.value, ms.value, by.value

    def tune_report(self) -> str:
        return _lib.swf_tune_report(self._ctx).decode()

    def reset_stats(self):
        self._check(_lib.swf_reset_stats(self._ctx))
