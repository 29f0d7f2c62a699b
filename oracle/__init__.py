"""CPU oracle for the AMHMVS checkerboard PatchMatch pass (arXiv 1805.07920).

TEST INFRASTRUCTURE ONLY.  A plain double-precision restatement of the
method (C, in ``amh_oracle.c``) plus this ctypes wrapper.  Only the tests,
the smoke check and the benchmark's CPU-baseline leg may import it; the GPU
library neither imports nor links it, and this module imports nothing from
the library.

The C header lists which functions are pinned by the tests and by what.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from dataclasses import dataclass

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
MAX_SRC = 32
N_OFFSETS = 72
# gcc flags: optimised for the host it runs on, every floating-point operation rounded as written
CFLAGS = ["-O3", "-march=native", "-ffp-contract=off", "-std=gnu11", "-fopenmp"]


def _host_tag() -> str:
    """Short tag of this host's CPU (model and feature flags): a library built with -march=native
    on one machine is never loaded on another."""
    import hashlib

    model = flags = ""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name") and not model:
                    model = line.split(":", 1)[1].strip()
                elif line.startswith("flags") and not flags:
                    flags = line.split(":", 1)[1].strip()
    except OSError:
        pass
    return hashlib.sha1((model + "|" + flags).encode()).hexdigest()[:12]


LIB_PATH = os.path.join(HERE, "_build", f"liborc-{_host_tag()}.so")


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def build(verbose: bool = False) -> str:
    """Compile the oracle with gcc for this host (OpenMP over same-colour pixels)."""
    os.makedirs(os.path.dirname(LIB_PATH), exist_ok=True)
    tmp = LIB_PATH + f".{os.getpid()}.tmp"
    cmd = ["gcc", *CFLAGS, "-shared", "-fPIC", "-o", tmp, os.path.join(HERE, "amh_oracle.c"), "-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB_PATH)
    return LIB_PATH


class _Views(C.Structure):
    _fields_ = [("W", C.c_int), ("H", C.c_int), ("n_src", C.c_int),
                ("ref", C.POINTER(C.c_float)),
                ("src", C.POINTER(C.c_float) * MAX_SRC),
                ("srcW", C.c_int * MAX_SRC), ("srcH", C.c_int * MAX_SRC),
                ("Kref", C.c_double * 9), ("Rref", C.c_double * 9), ("tref", C.c_double * 3),
                ("Ksrc", (C.c_double * 9) * MAX_SRC), ("Rsrc", (C.c_double * 9) * MAX_SRC),
                ("tsrc", (C.c_double * 3) * MAX_SRC)]


class _Params(C.Structure):
    _fields_ = [("refine", C.c_int), ("include_self", C.c_int),
                ("d_min", C.c_double), ("d_max", C.c_double), ("sigma_color", C.c_double),
                ("sigma_spatial", C.c_double), ("tau_mc_init", C.c_double), ("alpha", C.c_double),
                ("beta", C.c_double), ("tau_up", C.c_double),
                ("n1", C.c_int), ("n2", C.c_int), ("k", C.c_int), ("seed", C.c_uint64),
                ("view_mode", C.c_int), ("prop_mode", C.c_int), ("bilateral_sq", C.c_int),
                ("sample_f32", C.c_int), ("cost_noise", C.c_double)]


class _State(C.Structure):
    _fields_ = [("plane", C.POINTER(C.c_double)), ("cost", C.POINTER(C.c_double)),
                ("S", C.POINTER(C.c_uint32)), ("v", C.POINTER(C.c_int32))]


MAX_ROWS = 21  # propagated rows (8, or 20 in the standard symmetric pattern) + the pixel's own


class Diag(C.Structure):
    """Rows 0..n_prop-1 are the propagated hypotheses, row n_prop the pixel's own plane."""
    _fields_ = [("mfinal", C.c_double * MAX_ROWS), ("M", (C.c_double * MAX_SRC) * MAX_ROWS),
                ("row_valid", C.c_int * MAX_ROWS), ("cand_index", C.c_int * (MAX_ROWS - 1)),
                ("w", C.c_double * MAX_SRC), ("S", C.c_uint32), ("v", C.c_int),
                ("chosen", C.c_int), ("cand_cost", C.c_double * 6), ("cand_plane", (C.c_double * 4) * 6),
                ("n_cand", C.c_int), ("robust", C.c_int), ("n_prop", C.c_int)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            build()
        L = C.CDLL(LIB_PATH)
        u64p = C.POINTER(C.c_uint64)
        dp = C.POINTER(C.c_double)
        ip = C.POINTER(C.c_int)
        L.orc_philox4x64_10.argtypes = [u64p, u64p, u64p]
        L.orc_u24.argtypes = [C.c_uint64]
        L.orc_u24.restype = C.c_double
        L.orc_acp_offsets.argtypes = [ip, ip, ip]
        L.orc_acp_offsets.restype = C.c_int
        L.orc_scp_offsets.argtypes = [ip, ip, ip]
        L.orc_scp_offsets.restype = C.c_int
        L.orc_sscp_offsets.argtypes = [ip, ip, ip]
        L.orc_sscp_offsets.restype = C.c_int
        L.orc_project.argtypes = [C.POINTER(_Views), C.c_double, C.c_double, dp, C.c_int, dp]
        L.orc_matching_cost.argtypes = [C.POINTER(_Views), C.POINTER(_Params), C.c_int, C.c_int, dp, C.c_int]
        L.orc_matching_cost.restype = C.c_double
        L.orc_tau.argtypes = [C.POINTER(_Params), C.c_int]
        L.orc_tau.restype = C.c_double
        L.orc_view_selection.argtypes = [C.POINTER(_Params), C.c_int, dp, ip, C.c_int, C.c_uint32, C.c_int,
                                         C.POINTER(C.c_uint32), ip, dp]
        L.orc_view_selection_rows.argtypes = [C.POINTER(_Params), C.c_int, dp, ip, C.c_int, C.c_int, C.c_uint32,
                                              C.c_int, C.POINTER(C.c_uint32), ip, dp]
        L.orc_random_plane.argtypes = [C.POINTER(_Views), C.POINTER(_Params), C.c_int, C.c_int, C.c_uint64,
                                       C.c_uint64, dp]
        L.orc_init.argtypes = [C.POINTER(_Views), C.POINTER(_Params), C.POINTER(_State)]
        L.orc_pass.argtypes = [C.POINTER(_Views), C.POINTER(_Params), C.POINTER(_State), C.c_int, C.c_int,
                               ip, C.c_int, C.c_double, C.POINTER(Diag)]
        L.orc_run.argtypes = [C.POINTER(_Views), C.POINTER(_Params), C.POINTER(_State), C.c_int]
        L.orc_depth_normal.argtypes = [C.POINTER(_Views), C.POINTER(_State), dp, dp]
        L.orc_num_threads.restype = C.c_int
        L.orc_set_num_threads.argtypes = [C.c_int]
        _lib = L
    return _lib


def _dptr(a):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _iptr(a):
    return a.ctypes.data_as(C.POINTER(C.c_int))


# --------------------------------------------------------------------------------------
# parameters (the paper's values for the matching cost and the view inference)
# --------------------------------------------------------------------------------------

@dataclass
class Params:
    d_min: float = 2.0
    d_max: float = 6.0
    refine: int = 1
    include_self: int = 1
    sigma_color: float = 3.0
    sigma_spatial: float = 30.0
    tau_mc_init: float = 0.8
    alpha: float = 90.0
    beta: float = 0.3
    tau_up: float = 1.2
    n1: int = 2
    n2: int = 3
    k: int = 4
    seed: int = 0
    view_mode: int = 0  # 1: plain mean over all views (static objective for the sweep pin); 2: heuristic best-k
    prop_mode: int = 0  # 1: symmetric checkerboard propagation, fast (ablation); 2: standard (20 rows)
    bilateral_sq: int = 0  # 1: squared colour difference and distance in the bilateral weight
    sample_f32: int = 0  # conditioning probe (not the method): 1 sample positions and values rounded to float32,
    #                      2 also the NCC's sums and moments in float32, 3 the sample values moved by the
    #                      first-order bound of that rounding, each in the direction that moves the cost to 1
    cost_noise: float = 0.0  # conditioning probe (not the method): deterministic cost offsets of this width

    def c(self) -> _Params:
        return _Params(self.refine, self.include_self, self.d_min, self.d_max, self.sigma_color,
                       self.sigma_spatial, self.tau_mc_init, self.alpha, self.beta, self.tau_up,
                       self.n1, self.n2, self.k, self.seed & 0xFFFFFFFFFFFFFFFF, self.view_mode,
                       self.prop_mode, self.bilateral_sq, self.sample_f32, self.cost_noise)


class Views:
    """Reference + sources as the oracle sees them (float32 copies of the pixel values)."""

    def __init__(self, images, cams):
        if len(images) - 1 > MAX_SRC:
            raise ValueError("at most 32 sources")
        self.images = [np.ascontiguousarray(np.asarray(im, dtype=np.float32)) for im in images]
        v = _Views()
        v.H, v.W = self.images[0].shape
        v.n_src = len(images) - 1
        v.ref = self.images[0].ctypes.data_as(C.POINTER(C.c_float))
        for j, im in enumerate(self.images[1:]):
            v.src[j] = im.ctypes.data_as(C.POINTER(C.c_float))
            v.srcH[j], v.srcW[j] = im.shape
        c0 = cams[0]
        v.Kref[:] = np.asarray(c0.K, np.float64).ravel().tolist()
        v.Rref[:] = np.asarray(c0.R, np.float64).ravel().tolist()
        v.tref[:] = np.asarray(c0.t, np.float64).ravel().tolist()
        for j, cj in enumerate(cams[1:]):
            v.Ksrc[j][:] = np.asarray(cj.K, np.float64).ravel().tolist()
            v.Rsrc[j][:] = np.asarray(cj.R, np.float64).ravel().tolist()
            v.tsrc[j][:] = np.asarray(cj.t, np.float64).ravel().tolist()
        self.c = v
        self.W, self.H, self.n_src = v.W, v.H, v.n_src

    @classmethod
    def from_scene(cls, scene):
        return cls(scene.images, scene.cams)


@dataclass
class State:
    plane: np.ndarray  # (H, W, 4) float64
    cost: np.ndarray  # (H, W) float64
    S: np.ndarray  # (H, W) uint32
    v: np.ndarray  # (H, W) int32

    @classmethod
    def empty(cls, H, W):
        return cls(np.zeros((H, W, 4)), np.zeros((H, W)), np.zeros((H, W), np.uint32), np.full((H, W), -1, np.int32))

    @classmethod
    def from_arrays(cls, plane, cost, S, v):
        return cls(np.ascontiguousarray(plane, np.float64), np.ascontiguousarray(cost, np.float64),
                   np.ascontiguousarray(S, np.uint32), np.ascontiguousarray(v, np.int32))

    def copy(self):
        return State(self.plane.copy(), self.cost.copy(), self.S.copy(), self.v.copy())

    def c(self) -> _State:
        return _State(_dptr(self.plane), _dptr(self.cost), self.S.ctypes.data_as(C.POINTER(C.c_uint32)),
                      self.v.ctypes.data_as(C.POINTER(C.c_int32)))


# --------------------------------------------------------------------------------------
# functions
# --------------------------------------------------------------------------------------

def philox4x64_10(ctr, key) -> np.ndarray:
    c = np.array(ctr, dtype=np.uint64)
    k = np.array(key, dtype=np.uint64)
    o = np.zeros(4, np.uint64)
    p = C.POINTER(C.c_uint64)
    lib().orc_philox4x64_10(c.ctypes.data_as(p), k.ctypes.data_as(p), o.ctypes.data_as(p))
    return o


def u24(w: int) -> float:
    return lib().orc_u24(C.c_uint64(int(w)))


def acp_offsets():
    dx = np.zeros(N_OFFSETS, np.int32)
    dy = np.zeros(N_OFFSETS, np.int32)
    reg = np.zeros(N_OFFSETS, np.int32)
    n = lib().orc_acp_offsets(_iptr(dx), _iptr(dy), _iptr(reg))
    return dx[:n], dy[:n], reg[:n]


def scp_offsets():
    dx = np.zeros(8, np.int32)
    dy = np.zeros(8, np.int32)
    reg = np.zeros(8, np.int32)
    n = lib().orc_scp_offsets(_iptr(dx), _iptr(dy), _iptr(reg))
    return dx[:n], dy[:n], reg[:n]


def sscp_offsets():
    dx = np.zeros(N_OFFSETS, np.int32)
    dy = np.zeros(N_OFFSETS, np.int32)
    reg = np.zeros(N_OFFSETS, np.int32)
    n = lib().orc_sscp_offsets(_iptr(dx), _iptr(dy), _iptr(reg))
    return dx[:n], dy[:n], reg[:n]


def project(views: Views, sx: float, sy: float, plane, j: int) -> np.ndarray:
    pl = np.ascontiguousarray(plane, np.float64)
    out = np.zeros(3)
    lib().orc_project(C.byref(views.c), sx, sy, _dptr(pl), j, _dptr(out))
    return out


def matching_cost(views: Views, params: Params, x: int, y: int, plane, j: int) -> float:
    pl = np.ascontiguousarray(plane, np.float64)
    return lib().orc_matching_cost(C.byref(views.c), C.byref(params.c()), x, y, _dptr(pl), j)


def tau(params: Params, t: int) -> float:
    return lib().orc_tau(C.byref(params.c()), t)


def view_selection(params: Params, t: int, M, row_valid, S_prev: int = 0, v_prev: int = -1):
    """M: (R, N) costs of R propagated rows; R = 8 calls orc_view_selection, any other R
    orc_view_selection_rows (counts n1, n2 compared as fractions n R / 8 of the rows)."""
    M = np.ascontiguousarray(M, np.float64)
    R, N = M.shape
    assert 1 <= R <= MAX_ROWS - 1
    rv = np.ascontiguousarray(row_valid, np.int32)
    S = C.c_uint32(0)
    v = C.c_int(0)
    w = np.zeros(N)
    if R == 8:
        lib().orc_view_selection(C.byref(params.c()), t, _dptr(M), _iptr(rv), N, S_prev, v_prev, C.byref(S),
                                 C.byref(v), _dptr(w))
    else:
        lib().orc_view_selection_rows(C.byref(params.c()), t, _dptr(M), _iptr(rv), R, N, S_prev, v_prev,
                                      C.byref(S), C.byref(v), _dptr(w))
    return int(S.value), int(v.value), w


def random_plane(views: Views, params: Params, x: int, y: int, t: int = 0, purpose: int = 0) -> np.ndarray:
    out = np.zeros(4)
    lib().orc_random_plane(C.byref(views.c), C.byref(params.c()), x, y, t, purpose, _dptr(out))
    return out


def init(views: Views, params: Params) -> State:
    s = State.empty(views.H, views.W)
    cs = s.c()
    lib().orc_init(C.byref(views.c), C.byref(params.c()), C.byref(cs))
    return s


def run_pass(views: Views, params: Params, state: State, t: int, colour: int, order=None,
             delta: float = 0.0, diag: bool = False):
    """One half-pass in place.  ``order``: flat pixel indices to update (others untouched)."""
    cs = state.c()
    if order is None:
        lib().orc_pass(C.byref(views.c), C.byref(params.c()), C.byref(cs), t, colour, None, 0, delta, None)
        return None
    order = np.ascontiguousarray(order, np.int32)
    dg = (Diag * len(order))() if diag else None
    lib().orc_pass(C.byref(views.c), C.byref(params.c()), C.byref(cs), t, colour, _iptr(order), len(order), delta, dg)
    return dg


def run(views: Views, params: Params, iters: int) -> State:
    s = State.empty(views.H, views.W)
    cs = s.c()
    lib().orc_run(C.byref(views.c), C.byref(params.c()), C.byref(cs), iters)
    return s


def depth_normal(views: Views, state: State):
    d = np.zeros((views.H, views.W))
    n = np.zeros((views.H, views.W, 3))
    cs = state.c()
    lib().orc_depth_normal(C.byref(views.c), C.byref(cs), _dptr(d), _dptr(n))
    return d, n


def num_threads() -> int:
    return lib().orc_num_threads()


def set_num_threads(n: int) -> None:
    """OpenMP threads of the following oracle calls (the CPU baseline's one-core figure)."""
    lib().orc_set_num_threads(int(n))
