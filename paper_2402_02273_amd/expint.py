"""Python binding of the exponential-integrator library.

``ExpInt`` wraps one ``expint_ctx``: a grid, a diffusivity field, rho, the
boundary condition, the time step and the (s, m) plan.  Fields are torch
tensors on the GPU (z fastest, shape (nx, ny, nz)); this module only moves
pointers and checks shapes and dtypes on the host before each call.  All
arithmetic happens in the HIP library.
"""

from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import numpy as np
import torch

from . import _native as N

_DTYPES = {torch.float64: N.F64, torch.float32: N.F32}
_BCS = {"noflux": N.NOFLUX, "dirichlet0": N.DIRICHLET0}
_ALGOS = {"auto": N.ALGO_AUTO, "stencil_taylor": N.ALGO_STENCIL_TAYLOR, "modal": N.ALGO_MODAL}
_MPS = {"none": N.MP_NONE, "bf16_split": N.MP_BF16_SPLIT, "fp16_split": N.MP_FP16_SPLIT}
_SWEEPS = {"auto": N.SWEEPS_AUTO, "single": N.SWEEPS_SINGLE, "pairs": N.SWEEPS_PAIRS}
_SCHEMES = {"exp_euler": N.SCHEME_EXP_EULER, "linearised": N.SCHEME_LINEARISED, "exprk2": N.SCHEME_EXPRK2}


@dataclass
class Plan:
    s: int
    m: int
    norm_A1: float

    @property
    def terms(self) -> int:
        return self.s * self.m


def _stream_handle(stream, device):
    if stream is None:
        stream = torch.cuda.current_stream(device)
    return ctypes.c_void_p(int(stream.cuda_stream) or None)


def _as_device(x, device, dtype):
    t = torch.as_tensor(x)
    return t.to(device=device, dtype=dtype).contiguous()


class ExpInt:
    """One exponential integrator context on one GPU.

    scheme="exp_euler" steps u + tau phi1(tau A)(A u + f(u)); scheme="linearised"
    takes the paper's splitting of the reaction, u + tau phi1(tau J_n)(A u + f(u))
    with J_n = A + rho diag(1 - 2 u_n) (exponential Rosenbrock-Euler);
    scheme="exprk2" the second-order exponential Runge-Kutta step with phi2."""

    def __init__(
        self,
        shape,
        h: float = 1.0,
        *,
        labels=None,
        class_D=None,
        D=None,
        rho: float = 0.025,
        tau: float = 7.3,
        dtype=torch.float32,
        bc: str = "noflux",
        tol: float = 0.0,
        theta_max: float = 0.0,
        s: int = 0,
        m: int = 0,
        algo: str = "auto",
        mp: str = "none",
        check_finite: bool = False,
        sweeps: str = "auto",
        scheme: str = "exp_euler",
        device=None,
        stream=None,
    ):
        self.lib = N.lib()
        self.shape = tuple(int(v) for v in shape)
        if len(self.shape) != 3:
            raise ValueError("shape must be (nx, ny, nz)")
        device = torch.device("cuda") if device is None else torch.device(device)
        if device.type != "cuda":
            raise ValueError("the library runs on a GPU device")
        if device.index is None:
            device = torch.device("cuda", torch.cuda.current_device())
        self.device = device
        if dtype not in _DTYPES:
            raise ValueError("dtype must be torch.float32 or torch.float64")
        self.dtype = dtype
        self.n = int(np.prod(self.shape))
        self.h = float(h)
        self.tau = float(tau)
        self._ctx = ctypes.c_void_p()

        grid = N.Grid(self.shape[0], self.shape[1], self.shape[2], self.h)
        df = N.DField()
        keep = []
        if labels is not None:
            lab = _as_device(labels, self.device, torch.uint8)
            if lab.numel() != self.n:
                raise ValueError(f"labels hold {lab.numel()} voxels, grid has {self.n}")
            cd = (ctypes.c_double * len(class_D))(*[float(v) for v in class_D])
            keep += [lab, cd]
            df.labels = lab.data_ptr()
            df.n_classes = len(class_D)
            df.class_D = ctypes.cast(cd, ctypes.POINTER(ctypes.c_double))
            self.n_classes = len(class_D)
            self.class_D = tuple(float(v) for v in class_D)
        elif D is not None:
            Dt = _as_device(D, self.device, dtype)
            if Dt.numel() != self.n:
                raise ValueError(f"D holds {Dt.numel()} voxels, grid has {self.n}")
            keep.append(Dt)
            df.D = Dt.data_ptr()
            self.n_classes = 0
            self.class_D = None
        opts = N.Opts()
        N.check(self.lib.expint_opts_default(ctypes.byref(opts)))
        opts.dtype = _DTYPES[dtype]
        opts.tau = self.tau
        opts.tol = float(tol)
        opts.theta_max = float(theta_max)
        opts.algo = _ALGOS[algo]
        opts.mp = _MPS[mp]
        opts.s = int(s)
        opts.m = int(m)
        opts.check_finite = int(bool(check_finite))
        opts.sweeps = _SWEEPS[sweeps]
        opts.scheme = _SCHEMES[scheme]
        self.scheme = scheme
        with torch.cuda.device(self.device):
            opts.stream = _stream_handle(stream, self.device)
            N.check(
                self.lib.expint_create(
                    ctypes.byref(grid), ctypes.byref(df), float(rho), _BCS[bc], ctypes.byref(opts), ctypes.byref(self._ctx)
                )
            )
        self.rho = float(rho)
        self.bc = bc
        del keep

    # ---- lifetime ----
    def close(self):
        if getattr(self, "_ctx", None) and self._ctx.value:
            self.lib.expint_destroy(self._ctx)
            self._ctx = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    # ---- helpers ----
    def _field(self, t, name, writable=False):
        if not isinstance(t, torch.Tensor):
            raise TypeError(f"{name} must be a torch tensor")
        if t.device != self.device:
            raise ValueError(f"{name} is on {t.device}, context on {self.device}")
        if t.dtype != self.dtype:
            raise ValueError(f"{name} has dtype {t.dtype}, context uses {self.dtype}")
        if not t.is_contiguous() or t.numel() != self.n:
            raise ValueError(f"{name} must be contiguous with {self.n} elements")
        return ctypes.c_void_p(t.data_ptr())

    def empty(self):
        return torch.empty(self.shape, device=self.device, dtype=self.dtype)

    @property
    def stream(self) -> torch.cuda.ExternalStream:
        p = ctypes.c_void_p()
        N.check(self.lib.expint_get_stream(self._ctx, ctypes.byref(p)))
        if not p.value:
            return torch.cuda.default_stream(self.device)
        return torch.cuda.ExternalStream(p.value, device=self.device)

    # ---- plan and parameters ----
    def launch_info(self) -> dict:
        """The launch configuration resolved at creation (see expint_launch_info)."""
        li = N.LaunchInfo()
        N.check(self.lib.expint_get_launch(self._ctx, ctypes.byref(li)))
        return {f: getattr(li, f) for f, _ in N.LaunchInfo._fields_}

    def sweeps(self):
        """("single" or "pairs", pair tiling (ty, lp) or None) as resolved at creation."""
        li = self.launch_info()
        if li["sweeps"] == N.SWEEPS_PAIRS:
            return "pairs", (li["pair_ty"], li["pair_lp"])
        return "single", None

    @property
    def plan(self) -> Plan:
        s, m, nrm = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_double()
        N.check(self.lib.expint_get_plan(self._ctx, ctypes.byref(s), ctypes.byref(m), ctypes.byref(nrm)))
        return Plan(s.value, m.value, nrm.value)

    def set_params(self, rho=None, class_D=None, replan=True):
        rho = self.rho if rho is None else float(rho)
        cd = None
        if class_D is not None:
            cd = (ctypes.c_double * len(class_D))(*[float(v) for v in class_D])
        N.check(self.lib.expint_set_params(self._ctx, rho, cd, int(bool(replan))))
        self.rho = rho
        if class_D is not None:
            self.class_D = tuple(float(v) for v in class_D)

    # ---- operators ----
    def apply(self, x, out=None):
        out = self.empty() if out is None else out
        N.check(self.lib.expint_apply(self._ctx, self._field(x, "x"), self._field(out, "out")))
        return out

    def rhs(self, u, out=None):
        out = self.empty() if out is None else out
        N.check(self.lib.expint_rhs(self._ctx, self._field(u, "u"), self._field(out, "out")))
        return out

    def phi1(self, b, out=None):
        out = self.empty() if out is None else out
        N.check(self.lib.expint_phi1(self._ctx, self._field(b, "b"), self._field(out, "out")))
        return out

    def phi12(self, b, d, out=None):
        """tau phi1(tau A) b + tau phi2(tau A) d."""
        out = self.empty() if out is None else out
        N.check(self.lib.expint_phi12(self._ctx, self._field(b, "b"), self._field(d, "d"), self._field(out, "out")))
        return out

    def phi1_lin(self, u, b, out=None):
        """tau phi1(tau J) b with J = A + rho diag(1 - 2 u) (linearised contexts)."""
        out = self.empty() if out is None else out
        N.check(self.lib.expint_phi1_lin(self._ctx, self._field(u, "u"), self._field(b, "b"),
                                         self._field(out, "out")))
        return out

    def step(self, u):
        N.check(self.lib.expint_step(self._ctx, self._field(u, "u")))
        return u

    def advance_volumes(self, u, nsteps: int) -> np.ndarray:
        """nsteps steps in place; the tumour volume sum(u) / N after each."""
        vol = np.zeros(max(int(nsteps), 0), dtype=np.float64)
        ptr = vol.ctypes.data_as(ctypes.POINTER(ctypes.c_double)) if len(vol) else None
        N.check(self.lib.expint_advance_volumes(self._ctx, self._field(u, "u"), int(nsteps), ptr))
        return vol

    def tumour_size(self, u, threshold: float):
        """(d2, (a, b)): the largest squared distance in grid steps between
        two points with u > threshold and the smallest pair of linear indices
        reaching it."""
        d2 = ctypes.c_int64()
        pair = (ctypes.c_int64 * 2)()
        N.check(self.lib.expint_tumour_size(self._ctx, self._field(u, "u"), float(threshold), ctypes.byref(d2), pair))
        return int(d2.value), (int(pair[0]), int(pair[1]))

    def advance(self, u, nsteps: int):
        N.check(self.lib.expint_advance(self._ctx, self._field(u, "u"), int(nsteps)))
        return u

    def reduce(self, op: str, x, y=None) -> float:
        code = {"sum": 0, "dot": 1, "maxabs": 2, "mean": 3}[op]
        out = ctypes.c_double()
        yp = self._field(y, "y") if y is not None else None
        N.check(self.lib.expint_reduce(self._ctx, code, self._field(x, "x"), yp, ctypes.byref(out)))
        return out.value

    def tumour_volume(self, u) -> float:
        """Sum of the density over the grid divided by the voxel count."""
        return self.reduce("mean", u)

    # ---- gradients ----
    def grad(self, u0, nsteps, u_target, ckpt_every=10):
        gu = self.empty()
        loss, grho = ctypes.c_double(), ctypes.c_double()
        gD = (ctypes.c_double * max(self.n_classes, 1))()
        N.check(
            self.lib.expint_grad(
                self._ctx,
                self._field(u0, "u0"),
                int(nsteps),
                self._field(u_target, "u_target"),
                int(ckpt_every),
                ctypes.byref(loss),
                self._field(gu, "grad_u0"),
                ctypes.byref(grho),
                gD,
            )
        )
        return loss.value, gu, grho.value, list(gD)[: self.n_classes]

    def vjp(self, u0, nsteps, gout, ckpt_every=10):
        gu = self.empty()
        grho = ctypes.c_double()
        gD = (ctypes.c_double * max(self.n_classes, 1))()
        N.check(
            self.lib.expint_vjp(
                self._ctx,
                self._field(u0, "u0"),
                int(nsteps),
                self._field(gout, "gout"),
                int(ckpt_every),
                self._field(gu, "grad_u0"),
                ctypes.byref(grho),
                gD,
            )
        )
        return gu, grho.value, list(gD)[: self.n_classes]

    # ---- measurement ----
    def profile(self, kernel="flush", reps=50) -> float:
        """Mean ms per launch of one sweep of the step schedule.

        kernel: "flush" (Taylor term adding a pair of terms to the running sum),
        "skip" (Taylor term writing only its term), "rhs", for modal
        contexts "mode_x" / "mode_z" (the pass along x as the step runs it /
        the forward pass along z: a dense mode product, or fast transforms), for
        contexts with pair sweeps "pair" (two terms in one sweep), after a
        gradient call "face" (the gradient's fused reverse sweep)."""
        ms = ctypes.c_double()
        kid = {"flush": 0, "skip": 1, "rhs": 2, "mode_x": 3, "mode_z": 4, "pair": 5, "face": 6}[kernel]
        N.check(self.lib.expint_profile(self._ctx, kid, int(reps), ctypes.byref(ms)))
        return ms.value


class ExpIntBatch:
    """Many independent label-form grids advanced together (one HIP graph per step).

    ``instances``: sequence of dicts with ``labels`` (uint8 (nx, ny, nz)),
    ``class_D``, ``rho`` and optionally ``h``.  Every instance gets its own
    (s, m) plan and tile shape; tau, dtype, boundary and tolerances are shared.
    """

    def __init__(
        self,
        instances,
        *,
        tau: float = 7.3,
        dtype=torch.float32,
        bc: str = "noflux",
        tol: float = 0.0,
        theta_max: float = 0.0,
        s: int = 0,
        m: int = 0,
        scheme: str = "exp_euler",
        device=None,
        stream=None,
    ):
        self.lib = N.lib()
        device = torch.device("cuda") if device is None else torch.device(device)
        if device.index is None:
            device = torch.device("cuda", torch.cuda.current_device())
        self.device = device
        if dtype not in _DTYPES:
            raise ValueError("dtype must be torch.float32 or torch.float64")
        self.dtype = dtype
        self.scheme = scheme
        count = len(instances)
        if count < 1:
            raise ValueError("empty batch")
        grids = (N.Grid * count)()
        dfs = (N.DField * count)()
        rhos = (ctypes.c_double * count)()
        keep = []
        self.shapes = []
        for i, inst in enumerate(instances):
            lab = _as_device(inst["labels"], device, torch.uint8)
            shape = tuple(int(v) for v in np.shape(inst["labels"]))
            if len(shape) != 3 or lab.numel() != int(np.prod(shape)):
                raise ValueError(f"instance {i}: labels must be a 3-D array")
            cd = (ctypes.c_double * len(inst["class_D"]))(*[float(v) for v in inst["class_D"]])
            keep += [lab, cd]
            grids[i] = N.Grid(shape[0], shape[1], shape[2], float(inst.get("h", 1.0)))
            dfs[i].labels = lab.data_ptr()
            dfs[i].n_classes = len(inst["class_D"])
            dfs[i].class_D = ctypes.cast(cd, ctypes.POINTER(ctypes.c_double))
            rhos[i] = float(inst["rho"])
            self.shapes.append(shape)
        opts = N.Opts()
        N.check(self.lib.expint_opts_default(ctypes.byref(opts)))
        opts.dtype = _DTYPES[dtype]
        opts.tau = float(tau)
        opts.tol = float(tol)
        opts.theta_max = float(theta_max)
        opts.s = int(s)
        opts.m = int(m)
        opts.scheme = _SCHEMES[scheme]
        self._b = ctypes.c_void_p()
        with torch.cuda.device(device):
            opts.stream = _stream_handle(stream, device)
            N.check(
                self.lib.expint_batch_create(
                    count, grids, dfs, rhos, _BCS[bc], ctypes.byref(opts), ctypes.byref(self._b)
                )
            )
        self.count = count
        del keep

    def close(self):
        if getattr(self, "_b", None) and self._b.value:
            self.lib.expint_batch_destroy(self._b)
            self._b = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def plan(self, i) -> Plan:
        s, m, nrm = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_double()
        N.check(self.lib.expint_batch_get_plan(self._b, int(i), ctypes.byref(s), ctypes.byref(m), ctypes.byref(nrm)))
        return Plan(s.value, m.value, nrm.value)

    @property
    def plans(self):
        return [self.plan(i) for i in range(self.count)]

    def advance(self, us, nsteps: int):
        if len(us) != self.count:
            raise ValueError(f"{len(us)} fields for {self.count} instances")
        ptrs = (ctypes.c_void_p * self.count)()
        for i, (u, shape) in enumerate(zip(us, self.shapes)):
            if not isinstance(u, torch.Tensor) or u.device != self.device or u.dtype != self.dtype:
                raise ValueError(f"u[{i}] must be a {self.dtype} tensor on {self.device}")
            if not u.is_contiguous() or u.numel() != int(np.prod(shape)):
                raise ValueError(f"u[{i}] must be contiguous with {int(np.prod(shape))} elements")
            ptrs[i] = u.data_ptr()
        N.check(self.lib.expint_batch_advance(self._b, ptrs, int(nsteps)))
        return us


def labels_from_intensity(image, shape, thresholds=(1, 115, 240), stream=None, out=None):
    """uint8 labels on the stencil grid `shape` from a uint8 scan volume on a
    GPU (the thresholds of section 3.1 by default), into `out` if given."""
    if not isinstance(image, torch.Tensor) or image.dtype != torch.uint8 or image.dim() != 3:
        raise TypeError("image must be a 3-D torch.uint8 tensor")
    if image.device.type != "cuda":
        raise ValueError("image must be on a GPU")
    image = image.contiguous()
    shape = tuple(int(v) for v in shape)
    lab = torch.empty(shape, dtype=torch.uint8, device=image.device) if out is None else out
    if lab.dtype != torch.uint8 or tuple(lab.shape) != shape or not lab.is_contiguous() or lab.device != image.device:
        raise ValueError("out must be a contiguous uint8 tensor of the grid's shape on the image's device")
    th = (ctypes.c_int32 * len(thresholds))(*[int(v) for v in thresholds])
    lib = N.lib()
    with torch.cuda.device(image.device):
        st = _stream_handle(stream, image.device)
        N.check(lib.expint_labels_from_intensity(image.data_ptr(), *image.shape, th, len(thresholds), *shape,
                                                 lab.data_ptr(), st))
    return lab


def write_vtk(path, field, h: float = 1.0, name: str = "u", labels=None):
    """Writes `field` (and optionally `labels`) as a legacy VTK file for ParaView."""
    f = field.detach().cpu().numpy() if isinstance(field, torch.Tensor) else np.asarray(field)
    if f.ndim != 3 or f.dtype not in (np.float32, np.float64):
        raise TypeError("field must be a 3-D float32 or float64 array")
    f = np.ascontiguousarray(f)
    lab = None
    if labels is not None:
        lab = labels.detach().cpu().numpy() if isinstance(labels, torch.Tensor) else np.asarray(labels)
        if lab.shape != f.shape or lab.dtype != np.uint8:
            raise TypeError("labels must be uint8 with the field's shape")
        lab = np.ascontiguousarray(lab)
    dt = N.F64 if f.dtype == np.float64 else N.F32
    N.check(N.lib().expint_write_vtk(os.fsencode(path), *f.shape, float(h), f.ctypes.data, dt, name.encode(),
                                     None if lab is None else lab.ctypes.data))


def probe_peaks(device=None, hbm_bytes=1 << 30, cache_bytes=32 << 20, mfma_blocks=2048, mfma_iters=2048):
    """Attainable peaks of the device, measured by the library's probe kernels:
    copy bandwidth of an HBM-sized and of an Infinity-Cache-sized buffer
    (GB/s, bytes read + written) and the executed bf16 / fp16 matrix-core rate
    (TFLOP/s).  Allocates two buffers of hbm_bytes."""
    lib = N.lib()
    device = torch.device("cuda", torch.cuda.current_device()) if device is None else torch.device(device)
    out = {}
    with torch.cuda.device(device):
        st = torch.cuda.current_stream(device).cuda_stream
        a = torch.empty(hbm_bytes // 4, dtype=torch.float32, device=device).fill_(1.0)
        b = torch.empty_like(a)
        ms = ctypes.c_double()
        for name, nbytes, reps, nt in (("copy_hbm_GBs", hbm_bytes, 10, 1), ("copy_cache_GBs", cache_bytes, 200, 0)):
            N.check(lib.expint_probe_copy(a.data_ptr(), b.data_ptr(), int(nbytes), reps, nt, st, ctypes.byref(ms)))
            out[name] = 2.0 * nbytes / (ms.value * 1e-3) / 1e9
        del a, b
        sink = torch.empty(mfma_blocks * 256, dtype=torch.float32, device=device)
        tf = ctypes.c_double()
        for name, f16 in (("mfma_bf16_TFLOPs", 0), ("mfma_fp16_TFLOPs", 1)):
            N.check(lib.expint_probe_mfma(f16, mfma_iters, mfma_blocks, sink.data_ptr(), st, ctypes.byref(tf)))
            out[name] = tf.value
    out["note"] = (f"copy of {hbm_bytes >> 20} MiB (non-temporal) and {cache_bytes >> 20} MiB buffers "
                   f"(one 16-byte vector per lane); "
                   f"{mfma_blocks} x 4 waves x {mfma_iters} x 8 independent v_mfma_f32_32x32x16")
    return out
