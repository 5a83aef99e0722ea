"""Python binding of the apx C ABI (include/apx.h): argument marshalling only.

Every step of the hot path runs in the HIP library; PyTorch provides device memory and
the stream.  The binding raises if libapx.so is missing or no GPU is present -- there is
no CPU fallback.

Names follow the C entry points: render, chi2, jacobian, jtwj, chi2_grad, lm_init,
lm_step, lm_run.  ``Chi2Fn`` exposes chi^2 as a differentiable torch function whose
backward pass is the library's adjoint gradient.
"""
from __future__ import annotations

import ctypes
import os
from typing import Dict, List, Optional, Sequence

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libapx.so")

APX_OK, APX_E_INVALID, APX_E_HIP, APX_E_NONFINITE, APX_E_WORKSPACE, APX_E_UNSUPPORTED, APX_E_DOMAIN = \
    0, -1, -2, -3, -4, -5, -6
OBJECTIVE_FP64, OBJECTIVE_FP32 = 0, 1
CONV_DIRECT, CONV_FFT, CONV_DIRECT_2D, CONV_AUTO = 0, 1, 2, 3     # spec["conv_mode"]
SHIFT_NONE, SHIFT_BILINEAR, SHIFT_LANCZOS = 0, 1, 2   # spec["recentre"]["method"]

EXPORTS = [
    "apx_version", "apx_status_string", "apx_ctx_create", "apx_ctx_set_stream", "apx_ctx_destroy",
    "apx_last_error", "apx_problem_create", "apx_problem_workspace_bytes",
    "apx_problem_bind_workspace", "apx_problem_sizes", "apx_problem_check", "apx_problem_destroy",
    "apx_render", "apx_chi2", "apx_jacobian", "apx_jtwj", "apx_chi2_grad", "apx_render_vjp", "apx_lm_init",
    "apx_lm_step", "apx_lm_run", "apx_problem_set_timing", "apx_problem_timing",
    "apx_ctx_set_tiles", "apx_ctx_tile_cost", "apx_ctx_set_tile_cost", "apx_problem_tile_shapes", "apx_covariance",
    "apx_covariance_factor", "apx_hmc_run", "apx_nuts_run", "apx_nuts_warmup", "apx_problem_set_timing_classes",
    "apx_problem_set_wait_limit", "apx_problem_bind_scratch",
]
TILES_AUTOTUNE, TILES_MODEL, TILES_FIXED = 0, 1, 2
TILE_SHAPES = [(32, 64), (16, 64), (32, 32), (16, 32)]       # output rows x cols per workgroup
TIME_CLASSES = ["prep", "render", "conv_fwd", "deriv", "conv_jcol", "pairs", "reduce", "solve",
                "lm", "conv_adj", "grad", "conv_sep", "conv_fft"]


class ImageDesc(ctypes.Structure):
    _fields_ = [("H", ctypes.c_int32), ("W", ctypes.c_int32), ("P", ctypes.c_int32),
                ("sub", ctypes.c_int32), ("sky_par", ctypes.c_int32), ("psf_up", ctypes.c_int32),
                ("sky_fixed", ctypes.c_double), ("affine", ctypes.c_double * 6)]


class CompDesc(ctypes.Structure):
    _fields_ = [("type", ctypes.c_int32), ("image", ctypes.c_int32), ("box", ctypes.c_int32 * 4),
                ("par", ctypes.c_int32 * 7), ("reserved", ctypes.c_int32),
                ("fixed", ctypes.c_double * 7)]


class PsfModelDesc(ctypes.Structure):
    _fields_ = [("image", ctypes.c_int32), ("type", ctypes.c_int32), ("par", ctypes.c_int32 * 2),
                ("fixed", ctypes.c_double * 2)]


class ProblemDesc(ctypes.Structure):
    _fields_ = [("n_images", ctypes.c_int32), ("n_comps", ctypes.c_int32),
                ("n_par", ctypes.c_int32), ("n_sub", ctypes.c_int32),
                ("images", ctypes.POINTER(ImageDesc)), ("comps", ctypes.POINTER(CompDesc)),
                ("sub_par", ctypes.POINTER(ctypes.c_int32)), ("psf", ctypes.c_void_p),
                ("s", ctypes.c_int32), ("rule", ctypes.c_int32), ("mode", ctypes.c_int32),
                ("objective", ctypes.c_int32), ("k_re", ctypes.c_double),
                ("n_psf_models", ctypes.c_int32), ("conv_mode", ctypes.c_int32),
                ("psf_models", ctypes.POINTER(PsfModelDesc)),
                ("shift", ctypes.c_int32), ("shift_a", ctypes.c_int32)]


def _shift(spec: Dict):
    """(method, Lanczos order) of the spec's sub-pixel re-centring."""
    rc = spec.get("recentre")
    if not rc:
        return SHIFT_NONE, 0
    return int(rc["method"]), int(rc.get("a", 0))


PSF_MOFFAT = 0


def _psf_models(spec: Dict):
    """Live PSF models of the spec: entries dict(image, par=[n, R_d indices], fixed=[n, R_d])."""
    models = spec.get("psf_models", [])
    arr = (PsfModelDesc * max(1, len(models)))()
    for m, pm in enumerate(models):
        arr[m].image = int(pm["image"])
        arr[m].type = int(pm.get("type", PSF_MOFFAT))
        for q in range(2):
            arr[m].par[q] = int(pm["par"][q])
            arr[m].fixed[q] = float(pm["fixed"][q])
    return len(models), arr


class LMState(ctypes.Structure):
    _fields_ = [("lambda_", ctypes.c_double), ("chi2", ctypes.c_double),
                ("chi2_trial", ctypes.c_double), ("pred", ctypes.c_double),
                ("rho", ctypes.c_double), ("need_jac", ctypes.c_int32),
                ("accepted", ctypes.c_int32), ("n_accept", ctypes.c_int32),
                ("n_reject", ctypes.c_int32), ("n_chol_retry", ctypes.c_int32),
                ("status", ctypes.c_int32)]


LM_STATE_BYTES = ctypes.sizeof(LMState)
LM_STATE_DTYPE = np.dtype([("lambda", "<f8"), ("chi2", "<f8"), ("chi2_trial", "<f8"),
                           ("pred", "<f8"), ("rho", "<f8"), ("need_jac", "<i4"),
                           ("accepted", "<i4"), ("n_accept", "<i4"), ("n_reject", "<i4"),
                           ("n_chol_retry", "<i4"), ("status", "<i4")])
assert LM_STATE_DTYPE.itemsize == LM_STATE_BYTES


class ApxError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"apx status {status}: {msg}")
        self.status = status


_LIB = None


def check_buffer(t, device, dtype, numel: int, name: str):
    """Raise ApxError(APX_E_INVALID) unless t is a contiguous torch tensor of the given
    device, dtype and element count: a pointer handed to the library must be device memory
    of the size its kernels index."""
    import torch
    if not isinstance(t, torch.Tensor):
        raise ApxError(APX_E_INVALID, f"{name}: a torch tensor is required, got {type(t).__name__}")
    if t.device != device:
        raise ApxError(APX_E_INVALID, f"{name}: on {t.device}, the problem is on {device}")
    if t.dtype != dtype:
        raise ApxError(APX_E_INVALID, f"{name}: dtype {t.dtype}, {dtype} required")
    if not t.is_contiguous():
        raise ApxError(APX_E_INVALID, f"{name}: not contiguous")
    if t.numel() != numel:
        raise ApxError(APX_E_INVALID, f"{name}: {t.numel()} elements, {numel} required")
    return t


def load_library(path: str = LIB_PATH):
    """Load libapx.so (raises if it has not been built)."""
    global _LIB
    if _LIB is not None:
        return _LIB
    if not os.path.exists(path):
        raise ImportError(f"{path} is missing: build it with `python -m paper_2308_01957_amd.build`")
    lib = ctypes.CDLL(path)
    vp, i32, i64, u64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_uint64
    sig = {
        "apx_version": ([], ctypes.c_char_p),
        "apx_status_string": ([i32], ctypes.c_char_p),
        "apx_ctx_create": ([ctypes.c_int, vp, ctypes.POINTER(vp)], i32),
        "apx_ctx_set_stream": ([vp, vp], i32),
        "apx_ctx_destroy": ([vp], i32),
        "apx_last_error": ([vp], ctypes.c_char_p),
        "apx_problem_create": ([vp, ctypes.POINTER(ProblemDesc), ctypes.POINTER(vp)], i32),
        "apx_problem_workspace_bytes": ([vp, ctypes.POINTER(u64)], i32),
        "apx_problem_bind_workspace": ([vp, vp, u64], i32),
        "apx_problem_sizes": ([vp, ctypes.POINTER(i64), ctypes.POINTER(i64), ctypes.POINTER(i64)], i32),
        "apx_problem_check": ([vp], i32),
        "apx_problem_set_wait_limit": ([vp, i32], i32),
        "apx_problem_bind_scratch": ([vp], i32),
        "apx_problem_destroy": ([vp], i32),
        "apx_render": ([vp, vp, vp], i32),
        "apx_chi2": ([vp, vp, vp, vp, vp], i32),
        "apx_jacobian": ([vp, vp, vp, i64], i32),
        "apx_jtwj": ([vp, vp, vp, vp, vp, vp, vp], i32),
        "apx_chi2_grad": ([vp, vp, vp, vp, vp, vp], i32),
        "apx_render_vjp": ([vp, vp, vp, vp], i32),
        "apx_covariance": ([vp, vp, vp, vp, vp, vp], i32),
        "apx_covariance_factor": ([vp, vp, vp, vp, vp, vp], i32),
        "apx_hmc_run": ([vp, vp, vp, vp, vp, ctypes.c_double, i32, i32, vp, vp, vp, vp], i32),
        "apx_nuts_run": ([vp, vp, vp, vp, vp, ctypes.c_double, i32, i32, vp, vp, vp, vp], i32),
        "apx_nuts_warmup": ([vp, vp, vp, vp, vp, ctypes.POINTER(ctypes.c_double), i32, i32, ctypes.c_double,
                             vp, vp], i32),
        "apx_lm_init": ([vp, vp, vp, vp, vp], i32),
        "apx_lm_step": ([vp, vp, vp, vp, vp], i32),
        "apx_lm_run": ([vp, i32, vp, vp, vp, vp, i32], i32),
        "apx_problem_set_timing": ([vp, i32], i32),
        "apx_problem_set_timing_classes": ([vp, ctypes.c_uint32], i32),
        "apx_problem_timing": ([vp, i32, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(i64)], i32),
        "apx_ctx_set_tiles": ([vp, i32], i32),
        "apx_ctx_tile_cost": ([vp, i32, i32, ctypes.POINTER(ctypes.c_double)], i32),
        "apx_ctx_set_tile_cost": ([vp, i32, i32, ctypes.POINTER(ctypes.c_double)], i32),
        "apx_problem_tile_shapes": ([vp, i32, ctypes.POINTER(i32)], i32),
    }
    for name, (args, res) in sig.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = res
    _LIB = lib
    return lib


def _descs(spec: Dict):
    images = spec["images"]
    comps = spec["comps"]
    idesc = (ImageDesc * len(images))()
    for k, im in enumerate(images):
        d = idesc[k]
        d.H, d.W = int(im["H"]), int(im["W"])
        d.P = int(np.asarray(im["psf"]).shape[0])
        d.sub = int(im["sub"])
        d.sky_par = int(im["sky_par"])
        d.psf_up = int(im.get("up", 1))          # PSF samples per pixel per axis
        d.sky_fixed = float(im["sky_fixed"])
        for q in range(6):
            d.affine[q] = float(im["affine"][q])
    cdesc = (CompDesc * max(1, len(comps)))()
    for i, c in enumerate(comps):
        d = cdesc[i]
        d.type = int(c["type"])
        d.image = int(c["image"])
        for q in range(4):
            d.box[q] = int(c["box"][q])
        for q in range(7):
            d.par[q] = int(c["par"][q])
            d.fixed[q] = float(c["fixed"][q])
    sp = (ctypes.c_int32 * (2 * len(spec["subs"])))()
    for s, (p0, n) in enumerate(spec["subs"]):
        sp[2 * s], sp[2 * s + 1] = int(p0), int(n)
    return idesc, cdesc, sp


class Problem:
    """A model/fit problem bound to one GPU: descriptor, workspace and stream."""

    def __init__(self, spec: Dict, device: int = 0, objective: int = 0, tiles: int = TILES_AUTOTUNE,
                 tile_costs: Optional[Dict] = None, scratch: bool = False):
        """tile_costs: {(kernel, P): [us per tile of each shape]} entries of the autotuner's
        table to use instead of timing them (as read back by tile_cost()).  scratch: bind
        the library's own device scratch (apx_problem_bind_scratch) instead of allocating
        a workspace tensor."""
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("apx needs a ROCm GPU; none is visible")
        self.torch = torch
        self.lib = load_library()
        self.spec = spec
        self.device = torch.device("cuda", device)
        self.stream = torch.cuda.Stream(device=self.device)
        self.n_par = int(spec["n_par"])
        self.n_sub = len(spec["subs"])
        self.objective = int(objective)
        self.shapes = [(int(im["H"]), int(im["W"])) for im in spec["images"]]
        self.offsets = np.concatenate([[0], np.cumsum([h * w for h, w in self.shapes])]).astype(np.int64)
        self.n_pix = int(self.offsets[-1])
        psf = np.concatenate([np.ascontiguousarray(im["psf"], dtype=np.float32).ravel()
                              for im in spec["images"]])
        self.psf = torch.from_numpy(psf).to(self.device)
        self._ctx = ctypes.c_void_p()
        self._check(self.lib.apx_ctx_create(device, ctypes.c_void_p(self.stream.cuda_stream),
                                            ctypes.byref(self._ctx)), ctx=False)
        self._check(self.lib.apx_ctx_set_tiles(self._ctx, int(tiles)))
        for (kernel, P), us in (tile_costs or {}).items():
            arr = (ctypes.c_double * 4)(*[float(u) for u in us])
            self._check(self.lib.apx_ctx_set_tile_cost(self._ctx, int(kernel), int(P), arr))
        idesc, cdesc, sp = _descs(spec)
        sampling = spec["sampling"]
        npm, pms = _psf_models(spec)
        desc = ProblemDesc(len(spec["images"]), len(spec["comps"]), self.n_par, self.n_sub,
                           idesc, cdesc, sp, ctypes.c_void_p(self.psf.data_ptr()),
                           int(sampling["s"]), int(sampling["rule"]), int(sampling["mode"]),
                           int(objective), float(sampling.get("k", 0.0)), npm,
                           int(spec.get("conv_mode", CONV_DIRECT)), pms, *_shift(spec))
        self._keep = (idesc, cdesc, sp, desc, pms)
        self._prob = ctypes.c_void_p()
        self._check(self.lib.apx_problem_create(self._ctx, ctypes.byref(desc), ctypes.byref(self._prob)))
        nbytes = ctypes.c_uint64()
        self._check(self.lib.apx_problem_workspace_bytes(self._prob, ctypes.byref(nbytes)))
        self.workspace_bytes = int(nbytes.value)
        if scratch:
            self.workspace = None
            self._check(self.lib.apx_problem_bind_scratch(self._prob))
        else:
            with torch.cuda.stream(self.stream):
                self.workspace = torch.empty(max(256, self.workspace_bytes), dtype=torch.uint8, device=self.device)
            self._check(self.lib.apx_problem_bind_workspace(self._prob, ctypes.c_void_p(self.workspace.data_ptr()),
                                                            self.workspace.numel()))
        a, b, c = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64()
        self._check(self.lib.apx_problem_sizes(self._prob, ctypes.byref(a), ctypes.byref(b), ctypes.byref(c)))
        self.n_ext, self.n_jac = int(b.value), int(c.value)
        self.par_sub = np.full(self.n_par, -1, dtype=np.int64)
        for s, (p0, n) in enumerate(spec["subs"]):
            self.par_sub[p0:p0 + n] = s
        self.a_offsets = np.concatenate([[0], np.cumsum([n * n for _, n in spec["subs"]])]).astype(np.int64)

    def tile_shapes(self, kind: int) -> List[int]:
        """Convolution jobs of kind (0 model, 1 Jacobian columns, 2 adjoint) per tile shape
        (TILE_SHAPES order), then the jobs in FFT mode, then the jobs run as two 1-D passes
        (rank-one stamps)."""
        counts = (ctypes.c_int32 * 6)()
        self._check(self.lib.apx_problem_tile_shapes(self._prob, int(kind), counts))
        return list(counts)

    def tile_cost(self, kernel: int, P: int):
        """Autotuner's microseconds per tile of each shape, or None if not timed."""
        us = (ctypes.c_double * 4)()
        if self.lib.apx_ctx_tile_cost(self._ctx, int(kernel), int(P), us) != APX_OK:
            return None
        return list(us)

    # ------------------------------------------------------------------ helpers
    def _check(self, status: int, ctx: bool = True):
        if status != APX_OK:
            msg = self.lib.apx_last_error(self._ctx).decode() if ctx and self._ctx else ""
            raise ApxError(status, msg or self.lib.apx_status_string(status).decode())

    def _enter(self, *tensors):
        cur = self.torch.cuda.current_stream(self.device)
        self.stream.wait_stream(cur)
        for t in tensors:
            if t is not None:
                t.record_stream(self.stream)

    def _pix(self, data, weight):
        t = self.torch
        check_buffer(data, self.device, t.float32, self.n_pix, "data")
        check_buffer(weight, self.device, t.float32, self.n_pix, "weight")

    def _lm_bufs(self, theta, state):
        t = self.torch
        check_buffer(theta, self.device, t.float64, self.n_par, "theta")
        check_buffer(state, self.device, t.uint8, self.n_sub * LM_STATE_BYTES, "state")

    def _leave(self):
        self.torch.cuda.current_stream(self.device).wait_stream(self.stream)

    def _dev(self, x, dtype):
        t = self.torch
        if isinstance(x, t.Tensor):
            if x.device != self.device or x.dtype != dtype or not x.is_contiguous():
                x = x.to(device=self.device, dtype=dtype).contiguous()
            return x
        return t.as_tensor(np.ascontiguousarray(x), dtype=dtype, device=self.device)

    def _theta(self, x):
        """theta as a contiguous FP64 tensor on the problem's device, of n_par entries."""
        th = self._dev(x, self.torch.float64)
        if th.numel() != self.n_par:
            raise ApxError(APX_E_INVALID, f"theta: {th.numel()} elements, {self.n_par} required")
        return th

    def pixels(self, arrays: Sequence[np.ndarray]):
        """Concatenate per-image arrays into one FP32 device pixel buffer."""
        flat = np.concatenate([np.ascontiguousarray(a, dtype=np.float32).ravel() for a in arrays])
        return self.torch.from_numpy(flat).to(self.device)

    def split(self, flat) -> List[np.ndarray]:
        arr = flat.detach().cpu().numpy() if hasattr(flat, "detach") else np.asarray(flat)
        return [arr[self.offsets[k]:self.offsets[k + 1]].reshape(h, w) for k, (h, w) in enumerate(self.shapes)]

    def check(self):
        """Synchronise and raise if the device flagged an out-of-domain or non-finite input."""
        self._check(self.lib.apx_problem_check(self._prob))

    def synchronize(self):
        self.stream.synchronize()

    def set_wait_limit(self, polls: int):
        """Bound of the damped solve's hand-off waits (0: default; < 0: flags taken as never
        raised, every wait gives up after -polls polls and its step is dropped)."""
        self._check(self.lib.apx_problem_set_wait_limit(self._prob, int(polls)))

    # ----------------------------------------------------------------- hot path
    def render(self, theta, out=None):
        th = self._theta(theta)
        self._enter(th)
        with self.torch.cuda.stream(self.stream):
            if out is None:
                out = self.torch.empty(self.n_pix, dtype=self.torch.float32, device=self.device)
            check_buffer(out, self.device, self.torch.float32, self.n_pix, "out")
            self._check(self.lib.apx_render(self._prob, th.data_ptr(), out.data_ptr()))
        self._leave()
        return out

    def chi2(self, theta, data, weight, out=None):
        th = self._theta(theta)
        self._pix(data, weight)
        self._enter(th, data, weight)
        with self.torch.cuda.stream(self.stream):
            if out is None:
                out = self.torch.empty(self.n_sub, dtype=self.torch.float64, device=self.device)
            check_buffer(out, self.device, self.torch.float64, self.n_sub, "out")
            self._check(self.lib.apx_chi2(self._prob, th.data_ptr(), data.data_ptr(), weight.data_ptr(),
                                          out.data_ptr()))
        self._leave()
        return out

    def jacobian(self, theta):
        """Dense J as a (n_par, n_pix) FP32 tensor (row k = d model / d theta_k)."""
        th = self._theta(theta)
        self._enter(th)
        with self.torch.cuda.stream(self.stream):
            J = self.torch.empty((self.n_par, self.n_pix), dtype=self.torch.float32, device=self.device)
            self._check(self.lib.apx_jacobian(self._prob, th.data_ptr(), J.data_ptr(), self.n_pix))
        self._leave()
        return J

    def jtwj(self, theta, data, weight):
        """(JtWJ flat per-sub blocks, JtWr [n_par], chi2 [n_sub]), FP64 device tensors."""
        th = self._theta(theta)
        self._pix(data, weight)
        self._enter(th, data, weight)
        t = self.torch
        with t.cuda.stream(self.stream):
            A = t.empty(int(self.a_offsets[-1]), dtype=t.float64, device=self.device)
            g = t.empty(self.n_par, dtype=t.float64, device=self.device)
            c2 = t.empty(self.n_sub, dtype=t.float64, device=self.device)
            self._check(self.lib.apx_jtwj(self._prob, th.data_ptr(), data.data_ptr(), weight.data_ptr(),
                                          A.data_ptr(), g.data_ptr(), c2.data_ptr()))
        self._leave()
        return A, g, c2

    def block(self, A, s: int):
        n = self.spec["subs"][s][1]
        return A[int(self.a_offsets[s]):int(self.a_offsets[s + 1])].reshape(n, n)

    def covariance(self, theta, data, weight):
        """((J^T W J)^{-1} flat per-sub blocks, chi2 [n_sub]), FP64 device tensors."""
        th = self._theta(theta)
        self._pix(data, weight)
        self._enter(th, data, weight)
        t = self.torch
        with t.cuda.stream(self.stream):
            C = t.empty(max(1, int(self.a_offsets[-1])), dtype=t.float64, device=self.device)
            c2 = t.empty(self.n_sub, dtype=t.float64, device=self.device)
            self._check(self.lib.apx_covariance(self._prob, th.data_ptr(), data.data_ptr(), weight.data_ptr(),
                                                C.data_ptr(), c2.data_ptr()))
        self._leave()
        return C, c2

    def covariance_factor(self, theta, data, weight):
        """(F flat per-sub blocks with F F^T = (J^T W J)^{-1}, chi2 [n_sub]), FP64 device tensors."""
        th = self._theta(theta)
        self._pix(data, weight)
        self._enter(th, data, weight)
        t = self.torch
        with t.cuda.stream(self.stream):
            F = t.empty(max(1, int(self.a_offsets[-1])), dtype=t.float64, device=self.device)
            c2 = t.empty(self.n_sub, dtype=t.float64, device=self.device)
            self._check(self.lib.apx_covariance_factor(self._prob, th.data_ptr(), data.data_ptr(),
                                                       weight.data_ptr(), F.data_ptr(), c2.data_ptr()))
        self._leave()
        return F, c2

    def hmc(self, theta, data, weight, F, step: float, n_leapfrog: int, z, u):
        """Hamiltonian Monte Carlo from theta (device FP64 [n_par], updated in place to the
        chain's last state) with inverse-mass factor F (flat per-sub blocks); z: [n_samples,
        n_par] standard normals, u: [n_samples, n_sub] uniforms.  Returns (samples
        [n_samples, n_par], stats [n_samples, n_sub, 3] = accepted, H0, H1)."""
        t = self.torch
        z = self._dev(z, t.float64)
        u = self._dev(u, t.float64)
        F = self._dev(F, t.float64)
        n_samples = int(z.numel() // max(1, self.n_par)) if self.n_par else int(u.numel() // max(1, self.n_sub))
        if z.numel() != n_samples * self.n_par or u.numel() != n_samples * self.n_sub:
            raise ValueError("z must hold n_samples x n_par and u n_samples x n_sub entries")
        if F.numel() < int(self.a_offsets[-1]):
            raise ValueError("F must hold the per-sub blocks (sum of n_s^2 entries)")
        self._pix(data, weight)
        check_buffer(theta, self.device, t.float64, self.n_par, "theta")
        self._enter(theta, data, weight, F, z, u)
        with t.cuda.stream(self.stream):
            samples = t.empty((n_samples, self.n_par), dtype=t.float64, device=self.device)
            stats = t.empty((n_samples, self.n_sub, 3), dtype=t.float64, device=self.device)
            self._check(self.lib.apx_hmc_run(self._prob, data.data_ptr(), weight.data_ptr(), theta.data_ptr(),
                                             F.data_ptr(), float(step), int(n_leapfrog), n_samples,
                                             z.data_ptr(), u.data_ptr(), samples.data_ptr(), stats.data_ptr()))
        self._leave()
        return samples, stats

    def nuts(self, theta, data, weight, F, step: float, max_depth: int, z, u):
        """No-U-Turn sampling from theta (device FP64 [n_par], updated in place to the last
        sample) with inverse-mass factor F (flat per-sub blocks); z: [n_samples, n_par]
        standard normals, u: [n_samples, 1 + max_depth + 2^(max_depth+1)] uniforms.  Returns
        (samples [n_samples, n_par], stats [n_samples, 4] = depth, leapfrog steps, points in
        the slice, divergent)."""
        t = self.torch
        z = self._dev(z, t.float64)
        u = self._dev(u, t.float64)
        F = self._dev(F, t.float64)
        nd = 1 + int(max_depth) + (1 << (int(max_depth) + 1))
        n_samples = int(u.numel() // nd)
        if u.numel() != n_samples * nd or z.numel() != n_samples * self.n_par:
            raise ValueError("z must hold n_samples x n_par and u n_samples x (1 + d + 2^(d+1)) entries")
        if F.numel() < int(self.a_offsets[-1]):
            raise ValueError("F must hold the per-sub blocks (sum of n_s^2 entries)")
        self._pix(data, weight)
        check_buffer(theta, self.device, t.float64, self.n_par, "theta")
        self._enter(theta, data, weight, F, z, u)
        with t.cuda.stream(self.stream):
            samples = t.empty((n_samples, self.n_par), dtype=t.float64, device=self.device)
            stats = t.empty((n_samples, 4), dtype=t.float64, device=self.device)
            self._check(self.lib.apx_nuts_run(self._prob, data.data_ptr(), weight.data_ptr(), theta.data_ptr(),
                                              F.data_ptr(), float(step), int(max_depth), n_samples,
                                              z.data_ptr(), u.data_ptr(), samples.data_ptr(), stats.data_ptr()))
        self._leave()
        return samples, stats

    def nuts_warmup(self, theta, data, weight, F, step0: float, max_depth: int, target: float, z, u) -> float:
        """len(z) NUTS warm-up transitions from theta (advanced in place) adapting the step by
        dual averaging toward the target acceptance; returns the adapted step."""
        t = self.torch
        z = self._dev(z, t.float64)
        u = self._dev(u, t.float64)
        F = self._dev(F, t.float64)
        nd = 1 + int(max_depth) + (1 << (int(max_depth) + 1))
        n = int(u.numel() // nd)
        if u.numel() != n * nd or z.numel() != n * self.n_par:
            raise ValueError("z must hold n x n_par and u n x (1 + d + 2^(d+1)) entries")
        step = ctypes.c_double(float(step0))
        self._pix(data, weight)
        check_buffer(theta, self.device, t.float64, self.n_par, "theta")
        self._enter(theta, data, weight, F, z, u)
        with t.cuda.stream(self.stream):
            self._check(self.lib.apx_nuts_warmup(self._prob, data.data_ptr(), weight.data_ptr(), theta.data_ptr(),
                                                 F.data_ptr(), ctypes.byref(step), int(max_depth), n,
                                                 float(target), z.data_ptr(), u.data_ptr()))
        self._leave()
        return float(step.value)

    def render_vjp(self, theta, grad_model, out=None):
        """sum_i grad_model[i] d model_i / d theta (FP64 [n_par]) by the adjoint pass."""
        th = self._theta(theta)
        gm = self._dev(grad_model, self.torch.float32)
        if gm.numel() != self.n_pix:
            raise ValueError(f"grad_model has {gm.numel()} entries, the render has {self.n_pix} pixels")
        self._enter(th, gm)
        t = self.torch
        with t.cuda.stream(self.stream):
            if out is None:
                out = t.empty(self.n_par, dtype=t.float64, device=self.device)
            self._check(self.lib.apx_render_vjp(self._prob, th.data_ptr(), gm.data_ptr(), out.data_ptr()))
        self._leave()
        return out

    def chi2_grad(self, theta, data, weight):
        th = self._theta(theta)
        self._pix(data, weight)
        self._enter(th, data, weight)
        t = self.torch
        with t.cuda.stream(self.stream):
            g = t.empty(self.n_par, dtype=t.float64, device=self.device)
            c2 = t.empty(self.n_sub, dtype=t.float64, device=self.device)
            self._check(self.lib.apx_chi2_grad(self._prob, th.data_ptr(), data.data_ptr(), weight.data_ptr(),
                                               g.data_ptr(), c2.data_ptr()))
        self._leave()
        return g, c2

    def lm_init(self, theta, data, weight, theta_out=None, state_out=None):
        """Returns (theta device copy, state device buffer) ready for lm_step / lm_run.
        theta_out / state_out reuse existing buffers (a captured graph keys on them)."""
        t = self.torch
        src = self._theta(theta)
        self._pix(data, weight)
        if theta_out is not None:
            check_buffer(theta_out, self.device, t.float64, self.n_par, "theta_out")
        if state_out is not None:
            check_buffer(state_out, self.device, t.uint8, self.n_sub * LM_STATE_BYTES, "state_out")
        self._enter(src, data, weight)
        with t.cuda.stream(self.stream):
            if theta_out is None:
                th = src.clone()
            else:
                th = theta_out
                th.copy_(src)
            state = state_out if state_out is not None else \
                t.zeros(self.n_sub * LM_STATE_BYTES, dtype=t.uint8, device=self.device)
            self._check(self.lib.apx_lm_init(self._prob, th.data_ptr(), data.data_ptr(), weight.data_ptr(),
                                             state.data_ptr()))
        self._leave()
        return th, state

    def lm_step(self, data, weight, theta, state):
        self._pix(data, weight)
        self._lm_bufs(theta, state)
        self._enter(data, weight, theta, state)
        with self.torch.cuda.stream(self.stream):
            self._check(self.lib.apx_lm_step(self._prob, data.data_ptr(), weight.data_ptr(), theta.data_ptr(),
                                             state.data_ptr()))
        self._leave()

    def lm_run(self, n_iter: int, data, weight, theta, state, use_graph: bool = False):
        self._pix(data, weight)
        self._lm_bufs(theta, state)
        self._enter(data, weight, theta, state)
        with self.torch.cuda.stream(self.stream):
            self._check(self.lib.apx_lm_run(self._prob, int(n_iter), data.data_ptr(), weight.data_ptr(),
                                            theta.data_ptr(), state.data_ptr(), 1 if use_graph else 0))
        self._leave()

    def set_timing(self, enabled: bool, classes=None):
        """Record kernel times (HIP events): every class, or only the named classes."""
        if classes is None or not enabled:
            self._check(self.lib.apx_problem_set_timing(self._prob, 1 if enabled else 0))
        else:
            mask = 0
            for c in classes:
                mask |= 1 << TIME_CLASSES.index(c)
            self._check(self.lib.apx_problem_set_timing_classes(self._prob, mask))

    def timing(self) -> Dict[str, tuple]:
        """{class: (total_ms, launches)} since timing was enabled (synchronises)."""
        out = {}
        for k, name in enumerate(TIME_CLASSES):
            ms, n = ctypes.c_double(), ctypes.c_int64()
            self._check(self.lib.apx_problem_timing(self._prob, k, ctypes.byref(ms), ctypes.byref(n)))
            out[name] = (float(ms.value), int(n.value))
        return out

    def lm_state(self, state) -> np.ndarray:
        return np.frombuffer(state.cpu().numpy().tobytes(), dtype=LM_STATE_DTYPE)

    def close(self):
        if getattr(self, "_prob", None):
            self.stream.synchronize()
            self.lib.apx_problem_destroy(self._prob)
            self._prob = None
        if getattr(self, "_ctx", None):
            self.lib.apx_ctx_destroy(self._ctx)
            self._ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Plan:
    """Host-only view of a problem (device -1): descriptor validation and plan sizes,
    no GPU needed.  Raises ApxError exactly as Problem would for a bad spec."""

    def __init__(self, spec: Dict, objective: int = 0, tiles: int = TILES_MODEL):
        self.lib = load_library()
        self._ctx = ctypes.c_void_p()
        st = self.lib.apx_ctx_create(-1, None, ctypes.byref(self._ctx))
        if st != APX_OK:
            raise ApxError(st, "host context")
        st = self.lib.apx_ctx_set_tiles(self._ctx, int(tiles))
        if st != APX_OK:
            self.lib.apx_ctx_destroy(self._ctx)
            self._ctx = None
            raise ApxError(st, "tile policy")
        idesc, cdesc, sp = _descs(spec)
        sampling = spec["sampling"]
        npm, pms = _psf_models(spec)
        desc = ProblemDesc(len(spec["images"]), len(spec["comps"]), int(spec["n_par"]), len(spec["subs"]),
                           idesc, cdesc, sp, None, int(sampling["s"]), int(sampling["rule"]),
                           int(sampling["mode"]), int(objective), float(sampling.get("k", 0.0)), npm,
                           int(spec.get("conv_mode", CONV_DIRECT)), pms, *_shift(spec))
        self._keep = (idesc, cdesc, sp, desc, pms)
        self._prob = ctypes.c_void_p()
        st = self.lib.apx_problem_create(self._ctx, ctypes.byref(desc), ctypes.byref(self._prob))
        if st != APX_OK:
            msg = self.lib.apx_last_error(self._ctx).decode()
            self.lib.apx_ctx_destroy(self._ctx)
            self._ctx = None
            raise ApxError(st, msg)
        nbytes = ctypes.c_uint64()
        self.lib.apx_problem_workspace_bytes(self._prob, ctypes.byref(nbytes))
        self.workspace_bytes = int(nbytes.value)
        a, b, c = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64()
        self.lib.apx_problem_sizes(self._prob, ctypes.byref(a), ctypes.byref(b), ctypes.byref(c))
        self.n_pix, self.n_ext, self.n_jac = int(a.value), int(b.value), int(c.value)

    def tile_shapes(self, kind: int) -> List[int]:
        """Convolution jobs of kind (0 model, 1 Jacobian columns, 2 adjoint) per tile shape
        (TILE_SHAPES order), then the jobs in FFT mode, then the jobs run as two 1-D passes
        (rank-one stamps)."""
        counts = (ctypes.c_int32 * 6)()
        st = self.lib.apx_problem_tile_shapes(self._prob, int(kind), counts)
        if st != APX_OK:
            raise ApxError(st, "tile shapes")
        return list(counts)

    def close(self):
        if getattr(self, "_prob", None):
            self.lib.apx_problem_destroy(self._prob)
            self._prob = None
        if getattr(self, "_ctx", None):
            self.lib.apx_ctx_destroy(self._ctx)
            self._ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _chi2_fn():
    import torch

    class Chi2Fn(torch.autograd.Function):
        """chi^2 per sub-problem as a differentiable function of theta.

        forward: apx_chi2.  backward: apx_chi2_grad (the adjoint pass), each sub-problem's
        gradient scaled by the incoming gradient of its chi^2."""

        @staticmethod
        def forward(ctx, theta, problem, data, weight):
            ctx.problem, ctx.data, ctx.weight = problem, data, weight
            ctx.save_for_backward(theta.detach())
            return problem.chi2(theta.detach(), data, weight).clone()

        @staticmethod
        def backward(ctx, grad_out):
            (theta,) = ctx.saved_tensors
            p = ctx.problem
            g, _ = p.chi2_grad(theta, ctx.data, ctx.weight)
            ps = torch.as_tensor(p.par_sub, device=g.device)
            scale = torch.where(ps >= 0, grad_out.to(g.dtype)[ps.clamp(min=0)], torch.zeros_like(g))
            return g * scale, None, None, None

    return Chi2Fn


_CHI2_FN = []


def _render_fn():
    import torch

    class RenderFn(torch.autograd.Function):
        """Model pixels [n_pix] (FP32) as a differentiable function of theta.

        forward: apx_render.  backward: apx_render_vjp (the adjoint pass)."""

        @staticmethod
        def forward(ctx, theta, problem):
            ctx.problem = problem
            ctx.save_for_backward(theta.detach())
            return problem.render(theta.detach()).clone()

        @staticmethod
        def backward(ctx, grad_out):
            (theta,) = ctx.saved_tensors
            g = ctx.problem.render_vjp(theta, grad_out.detach().to(torch.float32).contiguous())
            return g.to(theta.dtype), None

    return RenderFn


_RENDER_FN = []


def render_autograd(theta, problem: "Problem"):
    """Differentiable model pixels [n_pix] of theta (backward = the library's adjoint)."""
    if not _RENDER_FN:
        _RENDER_FN.append(_render_fn())
    return _RENDER_FN[0].apply(theta, problem)


def chi2_autograd(theta, problem: "Problem", data, weight):
    """Differentiable chi^2 [n_sub] of theta (backward = the library's adjoint)."""
    if not _CHI2_FN:
        _CHI2_FN.append(_chi2_fn())
    return _CHI2_FN[0].apply(theta, problem, data, weight)
