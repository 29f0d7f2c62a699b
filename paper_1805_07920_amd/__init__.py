"""Python binding of libamhmvs (include/amhmvs.h): argument marshalling only.

Every step of the method runs in the library's gfx950 kernels; this module
converts numpy arrays / torch tensors to pointers and checks return codes.
torch is used only for device memory and the stream.  If the compiled library
is missing the import of :func:`lib` fails loudly -- there is no fallback.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "_build", "libamhmvs.so")

AMH_OK, AMH_E_INVALID_ARG, AMH_E_OOM, AMH_E_HIP, AMH_E_STATE, AMH_E_UNSUPPORTED = 0, -1, -2, -3, -4, -5
AMH_F32, AMH_F16 = 0, 1
AMH_STATIC_MAX_PIXELS = 2621440  # largest reference of amh_run_checkerboard_static (include/amhmvs.h)

# every function the header declares (checked against include/amhmvs.h by the tests)
EXPORTS = [
    "amh_params_default", "amh_create", "amh_set_params", "amh_init_views", "amh_begin", "amh_init_hypotheses",
    "amh_pass", "amh_run_checkerboard", "amh_get_depth_normal_cost", "amh_get_state", "amh_set_state",
    "amh_score_fixed", "amh_run_batch", "amh_get_job_result", "amh_get_job_times", "amh_tune", "amh_get_stats",
    "amh_status_str", "amh_last_error", "amh_destroy",
    "amh_nn_param_count", "amh_nn_init", "amh_nn_get_params", "amh_nn_set_params", "amh_nn_get_grads",
    "amh_nn_forward", "amh_nn_backward", "amh_nn_adam_step", "amh_nn_save", "amh_nn_load", "amh_sweep_features",
    "amh_init_from_proposal", "amh_run_proposal", "amh_set_launch_config", "amh_run_batch_proposal",
    "amh_fusion_params_default", "amh_median_filter4", "amh_fuse", "amh_run_checkerboard_static",
    "amh_set_initial_hypotheses", "amh_nn_targets", "amh_probe_valu",
]
NET_CELL = 4  # reference pixels per proposal cell side
NET_IN, NET_OUT = 16, 5
# tile order {XCD bands, hardware} x job order {given, largest first} x tile rows {4, 2} x batch half-passes
# {one launch each, one persistent launch}
N_TUNE_CONFIGS = 16


class AmhError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"amhmvs status {status}: {msg}")
        self.status = status


class amh_camera(C.Structure):
    _fields_ = [("K", C.c_double * 9), ("R", C.c_double * 9), ("t", C.c_double * 3),
                ("width", C.c_int), ("height", C.c_int)]


class amh_image(C.Structure):
    _fields_ = [("data", C.c_void_p), ("width", C.c_int), ("height", C.c_int), ("pitch_elems", C.c_int64),
                ("dtype", C.c_int), ("on_device", C.c_int)]


class amh_params(C.Structure):
    _fields_ = [("refine", C.c_int), ("include_self", C.c_int), ("depth_min", C.c_float), ("depth_max", C.c_float),
                ("sigma_color", C.c_float), ("sigma_spatial", C.c_float), ("tau_mc_init", C.c_float),
                ("alpha", C.c_float), ("beta", C.c_float), ("tau_up", C.c_float), ("n1", C.c_int), ("n2", C.c_int),
                ("k", C.c_int), ("seed", C.c_uint64), ("timing", C.c_int), ("conf_min", C.c_float),
                ("sym_prop", C.c_int), ("heuristic_views", C.c_int), ("bilateral_squared", C.c_int),
                ("sweep_sources", C.c_int)]


class amh_stats(C.Structure):
    _fields_ = [("evals_total", C.c_uint64), ("evals_init", C.c_uint64), ("evals_propagation", C.c_uint64),
                ("evals_refine", C.c_uint64), ("n_passes", C.c_int), ("ms_per_pass", C.c_float * 64),
                ("ms_init", C.c_float), ("ms_fuse_kernels", C.c_float), ("n_fuse_kernels", C.c_int),
                ("fallback_pixels", C.c_uint64), ("evals_short", C.c_uint64), ("evals_init_short", C.c_uint64)]


class amh_fusion_params(C.Structure):
    _fields_ = [("f_eps", C.c_float), ("f_ang_deg", C.c_float), ("f_con", C.c_int)]


class amh_job(C.Structure):
    _fields_ = [("ref", C.c_int), ("srcs", C.POINTER(C.c_int)), ("n_src", C.c_int), ("iters", C.c_int)]


_lib = None


def lib():
    """The loaded C-ABI library; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with __graft_entry__.build() (no CPU fallback)")
        L = C.CDLL(LIB_PATH)
        vp, ip, fp = C.c_void_p, C.c_int, C.c_float
        L.amh_params_default.argtypes = [C.POINTER(amh_params)]
        L.amh_create.argtypes = [C.POINTER(vp), C.POINTER(amh_params), vp]
        L.amh_set_params.argtypes = [vp, C.POINTER(amh_params)]
        L.amh_init_views.argtypes = [vp, ip, C.POINTER(amh_image), C.POINTER(amh_camera), ip]
        L.amh_begin.argtypes = [vp, ip, C.POINTER(C.c_int), ip]
        L.amh_init_hypotheses.argtypes = [vp]
        L.amh_pass.argtypes = [vp, ip, ip]
        L.amh_run_checkerboard.argtypes = [vp, ip, C.POINTER(C.c_int), ip, ip]
        L.amh_run_checkerboard_static.argtypes = [vp, ip, C.POINTER(C.c_int), ip, ip, vp, vp, vp]
        L.amh_get_depth_normal_cost.argtypes = [vp, vp, vp, vp, ip]
        L.amh_get_state.argtypes = [vp, vp, vp, vp, vp, ip]
        L.amh_set_state.argtypes = [vp, vp, vp, vp, vp, ip]
        L.amh_score_fixed.argtypes = [vp, vp, vp, ip, vp, ip]
        L.amh_run_batch.argtypes = [vp, ip, C.POINTER(amh_job)]
        L.amh_get_job_result.argtypes = [vp, ip, vp, vp, vp, ip]
        L.amh_get_job_times.argtypes = [vp, ip, C.POINTER(C.c_float)]
        L.amh_tune.argtypes = [vp, ip, C.POINTER(amh_job), C.POINTER(C.c_int), C.POINTER(C.c_float)]
        L.amh_get_stats.argtypes = [vp, C.POINTER(amh_stats)]
        L.amh_status_str.argtypes = [ip]
        L.amh_status_str.restype = C.c_char_p
        L.amh_last_error.argtypes = [vp]
        L.amh_last_error.restype = C.c_char_p
        L.amh_destroy.argtypes = [vp]
        L.amh_destroy.restype = None
        L.amh_nn_param_count.argtypes = [C.POINTER(C.c_int64)]
        L.amh_nn_init.argtypes = [vp, C.c_uint64]
        L.amh_nn_get_params.argtypes = [vp, vp, C.c_int64]
        L.amh_nn_set_params.argtypes = [vp, vp, C.c_int64]
        L.amh_nn_get_grads.argtypes = [vp, vp, C.c_int64]
        L.amh_nn_forward.argtypes = [vp, vp, vp, ip, ip, ip, vp]
        L.amh_nn_backward.argtypes = [vp, vp, C.POINTER(C.c_float)]
        L.amh_nn_adam_step.argtypes = [vp, fp, fp, fp, fp]
        L.amh_nn_save.argtypes = [vp, C.c_char_p]
        L.amh_nn_load.argtypes = [vp, C.c_char_p]
        L.amh_sweep_features.argtypes = [vp, vp, vp]
        L.amh_init_from_proposal.argtypes = [vp, vp, ip, ip]
        L.amh_set_initial_hypotheses.argtypes = [vp, vp, vp, vp, ip]
        L.amh_nn_targets.argtypes = [vp, vp, vp, vp, ip, ip, vp]
        L.amh_run_proposal.argtypes = [vp, ip, C.POINTER(C.c_int), ip, ip]
        L.amh_set_launch_config.argtypes = [vp, ip]
        L.amh_run_batch_proposal.argtypes = [vp, ip, C.POINTER(amh_job)]
        L.amh_fusion_params_default.argtypes = [C.POINTER(amh_fusion_params)]
        L.amh_median_filter4.argtypes = [vp, vp, vp, ip, ip]
        L.amh_probe_valu.argtypes = [ip, ip, ip, C.POINTER(C.c_float)]
        L.amh_fuse.argtypes = [vp, ip, C.POINTER(C.c_int), C.POINTER(vp), C.POINTER(vp),
                               C.POINTER(amh_fusion_params), vp, vp, vp, C.c_int64, C.POINTER(C.c_int64)]
        _lib = L
    return _lib


PROBE_KINDS = ("v_fma_f32 (vector operands)", "v_fma_f32 (scalar operand)", "v_rcp_f32", "v_fract_f32",
               "v_cvt_flr_i32_f32", "v_med3_i32", "v_mad_u32_u24", "v_add_f32 (literal)")


def probe_valu(kind: int, blocks: int, iters: int) -> float:
    """Device milliseconds of amh_probe_valu's launch (16 * iters * blocks * 4 wave instructions of one kind)."""
    ms = C.c_float()
    rc = lib().amh_probe_valu(kind, blocks, iters, C.byref(ms))
    if rc != AMH_OK:
        raise AmhError(rc, f"amh_probe_valu: {lib().amh_status_str(rc).decode()}")
    return float(ms.value)


def params_default(**kw) -> amh_params:
    p = amh_params()
    rc = lib().amh_params_default(C.byref(p))
    if rc != AMH_OK:
        raise AmhError(rc, "amh_params_default")
    for k, v in kw.items():
        if not hasattr(p, k):
            raise AttributeError(k)
        setattr(p, k, v)
    return p


def _camera(cam) -> amh_camera:
    c = amh_camera()
    c.K[:] = np.asarray(cam.K, np.float64).ravel().tolist()
    c.R[:] = np.asarray(cam.R, np.float64).ravel().tolist()
    c.t[:] = np.asarray(cam.t, np.float64).ravel().tolist()
    c.width, c.height = int(cam.width), int(cam.height)
    return c


def _ptr(x):
    """(pointer, on_device) of a numpy array or torch tensor; None -> (None, 0)."""
    if x is None:
        return None, 0
    if isinstance(x, np.ndarray):
        if not x.flags["C_CONTIGUOUS"]:
            raise ValueError("arrays must be C-contiguous")
        return x.ctypes.data, 0
    import torch

    if isinstance(x, torch.Tensor):
        if not x.is_contiguous():
            raise ValueError("tensors must be contiguous")
        return x.data_ptr(), 1 if x.is_cuda else 0
    raise TypeError(f"unsupported buffer type {type(x)}")


def _current_stream():
    try:
        import torch

        if torch.cuda.is_available():
            return torch.cuda.current_stream().cuda_stream
    except Exception:
        pass
    return None


class Context:
    """One amh_ctx: registered views, the current reference and its per-pixel state."""

    def __init__(self, params: amh_params | None = None, stream=None, **kw):
        self.L = lib()
        self.p = params if params is not None else params_default(**kw)
        h = C.c_void_p()
        s = stream if stream is not None else _current_stream()
        rc = self.L.amh_create(C.byref(h), C.byref(self.p), s)
        if rc != AMH_OK:
            raise AmhError(rc, "amh_create: " + self.L.amh_status_str(rc).decode())
        self.h = h
        self._keep = []
        self.W = self.H = 0
        self.n_src = 0

    def close(self):
        if getattr(self, "h", None):
            self.L.amh_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def _check(self, rc, what):
        if rc != AMH_OK:
            raise AmhError(rc, f"{what}: {self.L.amh_last_error(self.h).decode()}")

    # --- calls of the C-ABI -----------------------------------------------------------
    def set_params(self, params: amh_params):
        self._check(self.L.amh_set_params(self.h, C.byref(params)), "amh_set_params")
        self.p = params

    def init_views(self, images, cams, store_as: int = AMH_F32):
        n = len(images)
        arr = (amh_image * n)()
        camarr = (amh_camera * n)()
        keep = []
        for i, (im, cam) in enumerate(zip(images, cams)):
            ptr, dev = _ptr(im)
            if dev:
                import torch

                dt = AMH_F16 if im.dtype == torch.float16 else AMH_F32
                if im.dtype not in (torch.float16, torch.float32):
                    raise TypeError("images must be float32 or float16")
            else:
                if im.dtype not in (np.float16, np.float32):
                    raise TypeError("images must be float32 or float16")
                dt = AMH_F16 if im.dtype == np.float16 else AMH_F32
            keep.append(im)
            H, W = im.shape
            arr[i] = amh_image(ptr, W, H, W, dt, dev)
            camarr[i] = _camera(cam)
        self._check(self.L.amh_init_views(self.h, n, arr, camarr, store_as), "amh_init_views")
        self._views_shape = [tuple(im.shape) for im in images]

    def begin(self, ref: int, srcs):
        s = (C.c_int * len(srcs))(*[int(v) for v in srcs])
        self._check(self.L.amh_begin(self.h, ref, s, len(srcs)), "amh_begin")
        self.H, self.W = self._views_shape[ref]
        self.n_src = len(srcs)

    def init_hypotheses(self):
        self._check(self.L.amh_init_hypotheses(self.h), "amh_init_hypotheses")

    def pass_(self, t: int, colour: int):
        self._check(self.L.amh_pass(self.h, t, colour), "amh_pass")

    def run_checkerboard(self, ref: int, srcs, iters: int):
        s = (C.c_int * len(srcs))(*[int(v) for v in srcs])
        self._check(self.L.amh_run_checkerboard(self.h, ref, s, len(srcs), iters), "amh_run_checkerboard")
        self.H, self.W = self._views_shape[ref]
        self.n_src = len(srcs)

    def run_checkerboard_static(self, ref: int, srcs, iters: int, depth=None, normal=None, cost=None):
        """amh_run_checkerboard_static: the allocation-free run; outputs are device tensors (or None)."""
        H, W = self._views_shape[ref]
        for x, per_px, name in ((depth, 1, "depth"), (normal, 3, "normal"), (cost, 1, "cost")):
            if x is not None and (x.numel() != H * W * per_px or str(x.dtype) != "torch.float32"):
                raise ValueError(f"{name} must be a float32 tensor of {H * W * per_px} elements")
        ptrs = [_ptr(x) for x in (depth, normal, cost)]
        if any(p is not None and d != 1 for p, d in ptrs):
            raise ValueError("the allocation-free run writes device buffers only")
        s = (C.c_int * len(srcs))(*[int(v) for v in srcs])
        self._check(self.L.amh_run_checkerboard_static(self.h, ref, s, len(srcs), iters, *[p for p, _ in ptrs]),
                    "amh_run_checkerboard_static")
        self.n_src = len(srcs)
        return depth, normal, cost

    def get_depth_normal_cost(self, depth=None, normal=None, cost=None):
        """Host numpy outputs by default; pass device tensors to fill them in place."""
        if depth is None and normal is None and cost is None:
            depth = np.zeros((self.H, self.W), np.float32)
            normal = np.zeros((self.H, self.W, 3), np.float32)
            cost = np.zeros((self.H, self.W), np.float32)
        ptrs = [_ptr(x) for x in (depth, normal, cost)]
        devs = {d for p, d in ptrs if p is not None}
        if len(devs) > 1:
            raise ValueError("outputs must all be host or all device")
        dev = devs.pop() if devs else 0
        self._check(self.L.amh_get_depth_normal_cost(self.h, ptrs[0][0], ptrs[1][0], ptrs[2][0], dev),
                    "amh_get_depth_normal_cost")
        return depth, normal, cost

    def get_state(self):
        P = (self.H, self.W)
        planes = np.zeros(P + (4,), np.float32)
        cost = np.zeros(P, np.float32)
        S = np.zeros(P, np.uint32)
        v = np.zeros(P, np.int32)
        self._check(self.L.amh_get_state(self.h, planes.ctypes.data, cost.ctypes.data, S.ctypes.data,
                                         v.ctypes.data, 0), "amh_get_state")
        return planes, cost, S, v

    def set_state(self, planes, cost, S, v):
        arrs = [np.ascontiguousarray(planes, np.float32), np.ascontiguousarray(cost, np.float32),
                np.ascontiguousarray(S, np.uint32), np.ascontiguousarray(v, np.int32)]
        self._check(self.L.amh_set_state(self.h, *[a.ctypes.data for a in arrs], 0), "amh_set_state")

    def score_fixed(self, planes, pix):
        planes = np.ascontiguousarray(planes, np.float32).reshape(-1, 4)
        pix = np.ascontiguousarray(pix, np.int32).reshape(-1, 2)
        Q = planes.shape[0]
        out = np.zeros((Q, self.n_src), np.float32)
        self._check(self.L.amh_score_fixed(self.h, planes.ctypes.data, pix.ctypes.data, Q, out.ctypes.data, 0),
                    "amh_score_fixed")
        return out

    @staticmethod
    def _jobs(jobs):
        arr = (amh_job * len(jobs))()
        keep = []
        for i, jb in enumerate(jobs):
            s = (C.c_int * len(jb["srcs"]))(*[int(v) for v in jb["srcs"]])
            keep.append(s)
            arr[i] = amh_job(int(jb["ref"]), s, len(jb["srcs"]), int(jb["iters"]))
        return arr, keep

    def run_batch(self, jobs):
        arr, keep = self._jobs(jobs)
        self._check(self.L.amh_run_batch(self.h, len(jobs), arr), "amh_run_batch")
        self._jobs_shape = [self._views_shape[int(jb["ref"])] for jb in jobs]

    def run_batch_proposal(self, jobs):
        """The batch with every job initialised from the learned proposal (network must be loaded)."""
        arr, keep = self._jobs(jobs)
        self._check(self.L.amh_run_batch_proposal(self.h, len(jobs), arr), "amh_run_batch_proposal")
        self._jobs_shape = [self._views_shape[int(jb["ref"])] for jb in jobs]

    def tune(self, jobs):
        """Autotune the launch configuration on this batch; returns (best, ms per configuration)."""
        arr, keep = self._jobs(jobs)
        best = C.c_int(-1)
        ms = (C.c_float * N_TUNE_CONFIGS)()
        self._check(self.L.amh_tune(self.h, len(jobs), arr, C.byref(best), ms), "amh_tune")
        self._jobs_shape = [self._views_shape[int(jb["ref"])] for jb in jobs]
        return int(best.value), list(ms)

    def set_launch_config(self, config: int):
        """Launch configuration 0..7 (tile order + 2 job order + 4 two-row tiles); results do not depend on it."""
        self._check(self.L.amh_set_launch_config(self.h, int(config)), "amh_set_launch_config")

    def get_job_times(self):
        n = len(self._jobs_shape)
        out = (C.c_float * n)()
        self._check(self.L.amh_get_job_times(self.h, n, out), "amh_get_job_times")
        return np.array(out[:], np.float64)

    def get_job_result(self, job: int, depth=None, normal=None, cost=None):
        H, W = self._jobs_shape[job]
        if depth is None and normal is None and cost is None:
            depth = np.zeros((H, W), np.float32)
            normal = np.zeros((H, W, 3), np.float32)
            cost = np.zeros((H, W), np.float32)
        ptrs = [_ptr(x) for x in (depth, normal, cost)]
        dev = max(d for _, d in ptrs)
        self._check(self.L.amh_get_job_result(self.h, job, ptrs[0][0], ptrs[1][0], ptrs[2][0], dev),
                    "amh_get_job_result")
        return depth, normal, cost

    def get_stats(self) -> dict:
        s = amh_stats()
        self._check(self.L.amh_get_stats(self.h, C.byref(s)), "amh_get_stats")
        return dict(evals_total=s.evals_total, evals_init=s.evals_init, evals_propagation=s.evals_propagation,
                    evals_refine=s.evals_refine, n_passes=s.n_passes,
                    ms_per_pass=list(s.ms_per_pass[:s.n_passes]), ms_init=s.ms_init,
                    ms_fuse_kernels=s.ms_fuse_kernels, n_fuse_kernels=s.n_fuse_kernels,
                    fallback_pixels=s.fallback_pixels, evals_short=s.evals_short,
                    evals_init_short=s.evals_init_short)

    # --- learned proposal ----------------------------------------------------------------
    @staticmethod
    def nn_param_count() -> int:
        n = C.c_int64()
        rc = lib().amh_nn_param_count(C.byref(n))
        if rc != AMH_OK:
            raise AmhError(rc, "amh_nn_param_count")
        return int(n.value)

    def nn_init(self, seed: int = 0):
        self._check(self.L.amh_nn_init(self.h, int(seed)), "amh_nn_init")

    def nn_get_params(self) -> np.ndarray:
        out = np.zeros(self.nn_param_count(), np.float32)
        self._check(self.L.amh_nn_get_params(self.h, out.ctypes.data, out.size), "amh_nn_get_params")
        return out

    def nn_set_params(self, theta):
        theta = np.ascontiguousarray(theta, np.float32)
        self._check(self.L.amh_nn_set_params(self.h, theta.ctypes.data, theta.size), "amh_nn_set_params")

    def nn_get_grads(self) -> np.ndarray:
        out = np.zeros(self.nn_param_count(), np.float32)
        self._check(self.L.amh_nn_get_grads(self.h, out.ctypes.data, out.size), "amh_nn_get_grads")
        return out

    def nn_forward(self, feats, q_ref, out=None):
        """feats: device bfloat16 (n, h, w, 16); q_ref: device float32 (n, h, w) sweep inverse depth.
        Returns device (n, h, w, 5) float32: depth, unit normal, confidence."""
        import torch

        if feats.dtype != torch.bfloat16 or not feats.is_cuda or feats.dim() != 4 or feats.shape[3] != NET_IN:
            raise ValueError("feats must be a device bfloat16 tensor (n, h, w, 16)")
        n, h, w, _ = feats.shape
        if q_ref.dtype != torch.float32 or not q_ref.is_cuda or tuple(q_ref.shape) != (n, h, w):
            raise ValueError("q_ref must be a device float32 tensor (n, h, w)")
        if out is None:
            out = torch.empty((n, h, w, NET_OUT), dtype=torch.float32, device=feats.device)
        self._check(self.L.amh_nn_forward(self.h, _ptr(feats)[0], _ptr(q_ref)[0], n, h, w, _ptr(out)[0]),
                    "amh_nn_forward")
        return out

    def nn_backward(self, target, want_loss: bool = True):
        """target: device float32 tensor (n, h, w, 6); returns the loss (host float) or None."""
        loss = C.c_float(0.0)
        self._check(self.L.amh_nn_backward(self.h, _ptr(target)[0], C.byref(loss) if want_loss else None),
                    "amh_nn_backward")
        return float(loss.value) if want_loss else None

    def nn_targets(self, depth, normal, cost, out=None):
        """amh_nn_targets: device maps (H, W), (H, W, 3), (H, W) -> device targets (h, w, 6)."""
        import torch

        H, W = depth.shape
        h4, w4 = 8 * -(-H // 32), 8 * -(-W // 32)
        if out is None:
            out = torch.empty((h4, w4, 6), dtype=torch.float32, device=depth.device)
        for t, n in ((depth, H * W), (normal, 3 * H * W), (cost, H * W), (out, h4 * w4 * 6)):
            if not (t.is_cuda and t.dtype == torch.float32 and t.is_contiguous() and t.numel() == n):
                raise ValueError("nn_targets takes contiguous float32 device tensors of the documented sizes")
        self._check(self.L.amh_nn_targets(self.h, depth.data_ptr(), normal.data_ptr(), cost.data_ptr(), W, H,
                                          out.data_ptr()), "amh_nn_targets")
        return out

    def nn_adam_step(self, lr: float, beta1: float = 0.9, beta2: float = 0.999, eps: float = 1e-8):
        self._check(self.L.amh_nn_adam_step(self.h, lr, beta1, beta2, eps), "amh_nn_adam_step")

    def nn_save(self, path: str):
        self._check(self.L.amh_nn_save(self.h, os.fsencode(path)), "amh_nn_save")

    def nn_load(self, path: str):
        self._check(self.L.amh_nn_load(self.h, os.fsencode(path)), "amh_nn_load")

    def sweep_features(self, out=None, q_ref=None):
        """Network input of the current reference on its grid of 4x4 cells (8 ceil(H/32) x 8 ceil(W/32)):
        (device bfloat16 (h4, w4, 16), device float32 (h4, w4) inverse depth of the winning sweep plane)."""
        import torch

        shape = (8 * -(-self.H // 32), 8 * -(-self.W // 32))
        if out is None:
            out = torch.empty(shape + (NET_IN,), dtype=torch.bfloat16, device="cuda")
        if q_ref is None:
            q_ref = torch.empty(shape, dtype=torch.float32, device="cuda")
        self._check(self.L.amh_sweep_features(self.h, _ptr(out)[0], _ptr(q_ref)[0]), "amh_sweep_features")
        return out, q_ref

    def init_from_proposal(self, pred):
        """pred: device float32 (h, w, 5) per-cell depth, normal, confidence."""
        h, w = int(pred.shape[0]), int(pred.shape[1])
        self._check(self.L.amh_init_from_proposal(self.h, _ptr(pred)[0], h, w), "amh_init_from_proposal")

    def set_initial_hypotheses(self, depth, normal, conf=None):
        """amh_set_initial_hypotheses: per-pixel depth (H, W), normal (H, W, 3) and optional confidence
        (H, W), all numpy (host) or all device tensors."""
        arrs = [depth, normal, conf]
        if isinstance(depth, np.ndarray):
            arrs = [None if a is None else np.ascontiguousarray(a, np.float32) for a in arrs]
        ptrs = [_ptr(a) for a in arrs]
        devs = {d for p, d in ptrs if p is not None}
        if len(devs) != 1:
            raise ValueError("inputs must all be host or all device")
        for a, per, name in ((arrs[0], 1, "depth"), (arrs[1], 3, "normal"), (arrs[2], 1, "conf")):
            if a is not None and (a.size if isinstance(a, np.ndarray) else a.numel()) != self.H * self.W * per:
                raise ValueError(f"{name} must hold {self.H * self.W * per} values")
        self._check(self.L.amh_set_initial_hypotheses(self.h, ptrs[0][0], ptrs[1][0], ptrs[2][0], devs.pop()),
                    "amh_set_initial_hypotheses")

    def run_proposal(self, ref: int, srcs, iters: int):
        s = (C.c_int * len(srcs))(*[int(v) for v in srcs])
        self._check(self.L.amh_run_proposal(self.h, ref, s, len(srcs), iters), "amh_run_proposal")
        self.H, self.W = self._views_shape[ref]
        self.n_src = len(srcs)

    def median_filter4(self, src, dst=None):
        """4x4 median filter of a device float32 (H, W) depth map into dst (allocated if None)."""
        import torch

        if dst is None:
            dst = torch.empty_like(src)
        H, W = int(src.shape[0]), int(src.shape[1])
        self._check(self.L.amh_median_filter4(self.h, _ptr(src)[0], _ptr(dst)[0], W, H), "amh_median_filter4")
        return dst

    def fuse(self, views, depths, normals, f_eps: float = 0.3, f_ang_deg: float = 30.0, f_con: int = 2,
             capacity: int | None = None):
        """Point cloud of device depth (H, W) and normal (H, W, 3) maps of the registered ``views``:
        (points (P, 3), normals (P, 3), origin (P, 3) int32: view slot, pixel index, consistent views),
        device tensors trimmed to the P points fused."""
        import torch

        n = len(views)
        if len(depths) != n or len(normals) != n:
            raise ValueError("one depth and one normal map per view")
        if capacity is None:
            capacity = sum(int(d.numel()) for d in depths)
        pts = torch.empty((max(capacity, 1), 3), dtype=torch.float32, device="cuda")
        nrm = torch.empty_like(pts)
        org = torch.empty((max(capacity, 1), 3), dtype=torch.int32, device="cuda")
        v = (C.c_int * n)(*[int(x) for x in views])
        dp = (C.c_void_p * n)(*[_ptr(d)[0] for d in depths])
        np_ = (C.c_void_p * n)(*[_ptr(x)[0] for x in normals])
        fp = amh_fusion_params(f_eps, f_ang_deg, f_con)
        total = C.c_int64(0)
        self._check(self.L.amh_fuse(self.h, n, v, dp, np_, C.byref(fp), _ptr(pts)[0], _ptr(nrm)[0], _ptr(org)[0],
                                    capacity, C.byref(total)), "amh_fuse")
        k = min(int(total.value), capacity)
        return pts[:k], nrm[:k], org[:k], int(total.value)
